"""Benchmark of the TDSLDA step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-mixed] [--no-cpu]

One step = one AB4AM5 step (two right-hand-side evaluations, each with a
full density rebuild) of every evolved state.  The default workload is the
plain FP64 32^3 trapped gas with one vortex (32,768 evolved states, 65,536
represented); the FP32-mixed 48^3 run (8,192 evolved states) is reported in
the same JSON line under "fp32_mixed"; the batched quasi-1D, quasi-2D
(64x64, N_z = 64, 135,168 states) and warm-start experiments follow under
their own keys.  value = evolved states x steps / wall time of the timed
region (inputs resident in HBM, start-up excluded).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12  # MI355X HBM3E, bytes/s
COUNTERS_MD = os.path.join(ROOT, "profiles", "lap2_full_fp64_32_fp32_48_hbm_counters.md")


def algorithmic_bytes(kernel, S, nst, depth, fused=False, design=False):
    """Bytes a launch of each kernel moves for nst states of S bytes.

    Method bytes (default): what the step of Alg. AB4AM5 must move with the
    state on chip, 12 S per step: a density pass reads phi (1 S); the
    corrector pass reads phi and the partial corrector c and writes phi_new
    (3 S); the full pass reads phi and f_{k-1..k-D+1} and writes f_k, the
    next predictor p and partial corrector c (1 + (D - 1) + 3 = 7 S at
    D = 4).  The x-line pass of the split 3D Laplacian and the T = D2x phi
    read of the slab passes are this design's own traffic: 0 method bytes.
    design=True: the bytes the 3D kernels actually read and write once
    (T included: lap1 2 S, corrector 4 S, full pass 8 S).  The quasi-1D
    kernel set (fused=True) keeps each state in one lane group, so its
    design bytes are the method bytes."""
    method = {
        "dens": 1, "lap1": 0, "lap2_corr": 3, "lap2_f": 2, "lap2_h": 2,
        "lap2_full": 1 + (depth - 1) + 3,
        "pred": 1 + depth + 2,
        "lap2_taylor": 3, "norm": 1,
    }
    split = dict(method, lap1=2, lap2_corr=4, lap2_f=3, lap2_h=3, lap2_full=2 + (depth - 1) + 3, lap2_taylor=4)
    table = split if (design and not fused) else method
    return table[kernel] * S * nst if kernel in table else None


def design_rw(kernel, depth, fused=False):
    """(reads, writes) in units of S of one launch's design bytes (the
    bytes the kernel reads and writes once; see algorithmic_bytes)."""
    if fused:
        t = {"dens": (1, 0), "lap2_corr": (2, 1), "lap2_full": (1 + depth - 1, 3), "lap2_f": (1, 1),
             "pred": (1 + depth, 2)}
    else:
        t = {"dens": (1, 0), "lap1": (1, 1), "lap2_corr": (3, 1), "lap2_full": (2 + depth - 1, 3),
             "lap2_f": (2, 1), "lap2_h": (2, 1), "pred": (1 + depth, 2)}
    return t.get(kernel)


def stream_ceiling(reads, writes, read_bps, write_bps):
    """Rate (bytes/s) of a stream that reads `reads` and writes `writes`
    units when reads move at read_bps and writes at write_bps, one after the
    other per byte: (R + W) / (R / read_bps + W / write_bps)."""
    return (reads + writes) / (reads / read_bps + writes / write_bps)


def step_roofline(S):
    """Roofline state-steps/s of the method: 12 S per state-step at 8 TB/s."""
    return PEAK_HBM / (12.0 * S)


def run_workload(cfg, steps, warmup, seed_vortex, profile=True, precision=None, observe=False, A=1.0):
    import torch
    from paper_2602_08982_amd import tdslda as T
    from paper_2602_08982_amd import workloads as W
    import synth

    if cfg["name"].startswith("plain"):
        dx, dy = synth.vortex_offset(seed_vortex)
        vort = [(dx, dy, 1.0)]
    else:
        (x1, y1), (x2, y2) = synth.vortex_pair(seed_vortex)
        vort = [(x1, y1, 1.0), (x2, y2, -1.0)]
    stream = torch.cuda.current_stream().cuda_stream
    ctx, kidx = W.setup(cfg, vort, stream=stream, precision=precision, A=A)
    nst = len(kidx)
    t0 = time.time()
    ctx.abm_step(warmup)          # includes the Taylor start-up
    torch.cuda.synchronize()
    t_warm = time.time() - t0
    if profile:
        ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.abm_step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = ctx.kernel_stats() if profile else {}
    if profile:
        ctx.set_profiling(False)
    st, chk = ctx.check()
    obs = None
    if observe:
        d = ctx.densities()
        obs = dict(rho=d["rho"], nu=d["nu"], energy=ctx.energy())
    M = int(np.prod(cfg["n"]))
    prec = cfg["precision"] if precision is None else precision
    es = 16 if prec == T.FP64 else 8
    S = 2 * M * es
    depth = 4
    kern = {}
    for k, (n, ms) in stats.items():
        if n == 0:
            continue
        b = algorithmic_bytes(k, S, nst, depth)
        bd = algorithmic_bytes(k, S, nst, depth, design=True)
        avg = ms / n
        kern[k] = dict(launches=n, avg_ms=avg, total_ms=ms,
                       gbps=(b / (avg * 1e-3) / 1e9) if b else None,
                       design_gbps=(bd / (avg * 1e-3) / 1e9) if bd else None)
    ctx.close()
    del ctx
    return dict(nst=nst, seconds=dt, warm_seconds=t_warm, value=nst * steps / dt,
                ms_per_step=1e3 * dt / steps, kernels=kern, check=dict(status=st, **chk), S=S,
                vortices=vort, obs=obs)


def track_precision(steps, every, warmup, seed_vortex=4):
    """The FP32-mixed 48^3 workload and its FP64 run side by side in time
    (one after the other on the device): rho, nu and E of both every
    `every` steps after the warm-up; returns the relative errors of the
    FP32-mixed run at each checkpoint (not timed)."""
    from paper_2602_08982_amd import tdslda as T
    from paper_2602_08982_amd import workloads as W
    import synth
    (x1, y1), (x2, y2) = synth.vortex_pair(seed_vortex)
    vort = [(x1, y1, 1.0), (x2, y2, -1.0)]
    runs = {}
    for prec in (T.FP32_MIXED, T.FP64):
        ctx, _ = W.setup(W.MIXED, vort, precision=prec)
        ctx.abm_step(warmup)
        obs = []
        for done in range(every, steps + 1, every):
            ctx.abm_step(every)
            d = ctx.densities()
            obs.append((done, d["rho"], d["nu"], ctx.energy()))
        ctx.close()
        runs[prec] = obs
        print(f"# precision track: {'fp32-mixed' if prec == T.FP32_MIXED else 'fp64'} run done", file=sys.stderr,
              flush=True)
    out = []
    for (k, r32, n32, e32), (_, r64, n64, e64) in zip(runs[T.FP32_MIXED], runs[T.FP64]):
        out.append(dict(step=k, rho_rel_err=float(np.abs(r32 - r64).max() / np.abs(r64).max()),
                        nu_rel_err=float(np.abs(n32 - n64).max() / np.abs(n64).max()),
                        energy_rel_err=float(abs(e32["total"] - e64["total"]) / abs(e64["EFG"]))))
    return out


def run_q1d(steps, warmup, seed=7, profile_steps=2, friction=False, precision=None, A=1.0, eager=False):
    """Batched quasi-1D workload: set-up (device eigensolver), start-up and
    warm-up steps, launch-shape tuning, then `steps` steps recorded as one
    HIP graph and launched once (timed from launch to completion).
    friction: the same with the quantum-friction terms on (alpha = beta = 5,
    gamma = 0.1, rho0 = the initial maximum density, N_req = the initial N).
    precision: the context precision (default: the workload's FP32-mixed).
    A: the functional's A (1.094 = the general functional of Eq. h_sigma,
    evolving the same initial states).
    eager: time `steps` steps of tdslda_abm_step (one launch per kernel, no
    graph in the process) instead of the graph launch."""
    import torch
    from paper_2602_08982_amd import tdslda as T
    from paper_2602_08982_amd import workloads as W
    t0 = time.perf_counter()
    ctx, info = W.setup_q1d(W.Q1D, seed, stream=torch.cuda.current_stream().cuda_stream, precision=precision, A=A)
    t_setup = time.perf_counter() - t0
    nst = info["states"]
    prec = W.Q1D["precision"] if precision is None else precision
    S = 2 * W.Q1D["nz"] * (16 if prec == T.FP64 else 8)
    if friction:
        rho0 = float(ctx.densities()["rho"].max())
        ctx.set_friction(alpha=5.0, beta=5.0, gamma=0.1, rho0=rho0, N_req=ctx.energy()["N"])
    ctx.abm_step(warmup)
    tuned = ctx.autotune()
    torch.cuda.synchronize()
    if eager:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.abm_step(steps)
        torch.cuda.synchronize()
        rec_ms, dt = 0.0, time.perf_counter() - t0
    else:
        rec_ms, run_ms = ctx.abm_graph(steps)
        dt = run_ms * 1e-3
    kern = {}
    if profile_steps:
        ctx.set_profiling(True)
        ctx.abm_step(profile_steps)
        stats = ctx.kernel_stats()
        ctx.set_profiling(False)
        for k, (n, ms) in stats.items():
            if n == 0:
                continue
            b = algorithmic_bytes(k, S, nst, 4, fused=True)
            avg = ms / n
            kern[k] = dict(launches=n, avg_ms=avg, total_ms=ms, gbps=(b / (avg * 1e-3) / 1e9) if b else None)
    st, chk = ctx.check()
    ctx.close()
    info = {k: v for k, v in info.items() if k not in ("kperp2", "counts")}
    return dict(nst=nst, steps=steps, seconds=dt, value=nst * steps / dt, ms_per_step=1e3 * dt / steps,
                graph_record_ms=rec_ms, setup_seconds=t_setup, tuned=tuned, kernels=kern,
                profile_steps=profile_steps, S=S,
                check=dict(status=st, **chk), problems=info)


def run_q1d_aslda(steps, warmup, profile_steps=2, precision=None):
    """Spin-imbalanced batched quasi-1D workload (workloads.Q1D_ASLDA): both
    branches from the device eigensolver, start-up and warm-up, launch-shape
    tuning, then `steps` steps in one HIP-graph launch; the polarisation and
    the conservation check after the run."""
    import torch
    from paper_2602_08982_amd import tdslda as T
    from paper_2602_08982_amd import workloads as W
    t0 = time.perf_counter()
    ctx, info = W.setup_q1d_aslda(W.Q1D_ASLDA, stream=torch.cuda.current_stream().cuda_stream, precision=precision)
    t_setup = time.perf_counter() - t0
    nst = info["states"]
    prec = W.Q1D_ASLDA["precision"] if precision is None else precision
    S = 2 * W.Q1D_ASLDA["nz"] * (16 if prec == T.FP64 else 8)
    ctx.abm_step(warmup)
    tuned = ctx.autotune()
    rec_ms, run_ms = ctx.abm_graph(steps)
    dt = run_ms * 1e-3
    kern = {}
    if profile_steps:
        ctx.set_profiling(True)
        ctx.abm_step(profile_steps)
        stats = ctx.kernel_stats()
        ctx.set_profiling(False)
        for k, (n, ms) in stats.items():
            if n:
                kern[k] = dict(launches=n, avg_ms=ms / n, total_ms=ms)
    d = ctx.densities_spin()
    ra, rb = d["rho"]
    pol = float(((ra - rb) / np.maximum(ra + rb, 1e-30)).max())
    st, chk = ctx.check()
    ctx.close()
    return dict(nst=nst, steps=steps, seconds=dt, value=nst * steps / dt, ms_per_step=1e3 * dt / steps,
                setup_seconds=t_setup, tuned=tuned, kernels=kern, S=S, max_polarisation=pol,
                check=dict(status=st, **chk), problems=info)


def run_aslda3d(steps, warmup, profile_steps=1):
    """Spin-imbalanced 3D workload (workloads.ASLDA3D): both branches of the
    uniform start, start-up and warm-up, `steps` steps timed between two
    device synchronisations, then `profile_steps` with per-kernel events."""
    import torch
    from paper_2602_08982_amd import workloads as W
    t0 = time.perf_counter()
    ctx, kidx = W.setup_aslda3d(W.ASLDA3D, stream=torch.cuda.current_stream().cuda_stream)
    ctx.abm_step(warmup)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    nst = 2 * len(kidx)
    t0 = time.perf_counter()
    ctx.abm_step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern = {}
    if profile_steps:
        ctx.set_profiling(True)
        ctx.abm_step(profile_steps)
        for k, (n, ms) in ctx.kernel_stats().items():
            if n:
                kern[k] = dict(launches=n, avg_ms=ms / n, total_ms=ms)
        ctx.set_profiling(False)
    d = ctx.densities_spin()
    ra, rb = d["rho"]
    pol = float(((ra - rb) / np.maximum(ra + rb, 1e-30)).max())
    st, chk = ctx.check()
    ctx.close()
    return dict(nst=nst, steps=steps, seconds=dt, value=nst * steps / dt, ms_per_step=1e3 * dt / steps,
                setup_seconds=t_setup, kernels=kern, max_polarisation=pol, check=dict(status=st, **chk))


def run_q2d(steps, warmup, seed_vortex=2, profile_steps=2, precision=None):
    """Quasi-2D workload (workloads.Q2D): set-up, start-up and warm-up
    steps, then `steps` steps of tdslda_abm_step timed between two device
    synchronisations (one launch per kernel), then `profile_steps` more
    with per-kernel events."""
    import torch
    from paper_2602_08982_amd import tdslda as T
    from paper_2602_08982_amd import workloads as W
    import synth
    dx, dy = synth.vortex_offset(seed_vortex)
    vort = [(dx, dy, 1.0)]
    t0 = time.perf_counter()
    ctx, kidx = W.setup_q2d(W.Q2D, vort, stream=torch.cuda.current_stream().cuda_stream, precision=precision)
    ctx.abm_step(warmup)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    nst = len(kidx)
    prec = W.Q2D["precision"] if precision is None else precision
    M = W.Q2D["n"][0] * W.Q2D["n"][1]
    S = 2 * M * (16 if prec == T.FP64 else 8)
    t0 = time.perf_counter()
    ctx.abm_step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern = {}
    if profile_steps:
        ctx.set_profiling(True)
        ctx.abm_step(profile_steps)
        stats = ctx.kernel_stats()
        ctx.set_profiling(False)
        for k, (n, ms) in stats.items():
            if n == 0:
                continue
            b = algorithmic_bytes(k, S, nst, 4, fused=True)
            avg = ms / n
            kern[k] = dict(launches=n, avg_ms=avg, total_ms=ms, gbps=(b / (avg * 1e-3) / 1e9) if b else None)
    st, chk = ctx.check()
    e = ctx.energy()
    ctx.close()
    return dict(nst=nst, steps=steps, seconds=dt, value=nst * steps / dt, ms_per_step=1e3 * dt / steps,
                setup_seconds=t_setup, kernels=kern, profile_steps=profile_steps, S=S,
                check=dict(status=st, **chk), N=e["N"], vortices=vort)


def stream_rates():
    """This device's HBM stream rates from the library's own streaming
    kernels over 4 GiB (median of 5, HIP events on the launch stream):
    read = tdslda_device_read, copy = tdslda_device_copy (read + write
    bytes); the write rate follows from the two: a copy of B bytes takes
    (B/2)/read + (B/2)/write."""
    import torch
    from paper_2602_08982_amd import tdslda as T
    n = 1 << 29
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    sink = torch.zeros(2, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()

    def med(fn):
        fn()
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            fn()
            e1.record(st)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return sorted(ts)[2]
    t_copy = med(lambda: T.device_copy(b, a, 8 * n, st.cuda_stream))
    t_read = med(lambda: T.device_read(a, 8 * n, sink, st.cuda_stream))
    ok = bool(torch.equal(a, b))
    del a, b, sink
    torch.cuda.empty_cache()
    if not ok:
        raise RuntimeError("device copy produced wrong data")
    read = 8 * n / t_read
    copy = 2 * 8 * n / t_copy
    write = 0.5 / (1.0 / copy - 0.5 / read)
    return dict(read=read, copy=copy, write=write)


def roofline(res, rates=None, prec=None, nx=None, role_prefix="", fused=False):
    """Dominant kernel of the timed steps against the HBM peak.
    achieved = method bytes per launch (algorithmic_bytes) / mean launch
    time; the kernel's own read-once / write-once bytes (the split-Laplacian
    intermediate included) are reported beside it as design_*.
    step_frac = state-steps/s / the method's roofline rate 8 TB/s / (12 S).
    traffic = HBM bytes per launch from the committed FETCH_SIZE /
    WRITE_SIZE summary (copy-calibrated), null when that summary does not
    cover this kernel or the kernel sources changed since the counters
    were taken.  stream_ceiling = the rate this device's streaming kernels
    reach for the kernel's read / write mix (stream_rates, stream_ceiling),
    the measured ceiling its design bytes are compared with."""
    kern = res["kernels"]
    if not kern:
        return None
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    g = kern[dom]["gbps"]
    gd = kern[dom].get("design_gbps")
    avg_s = kern[dom]["avg_ms"] * 1e-3
    traffic = None
    if prec is not None:
        from paper_2602_08982_amd import profsum
        traffic = profsum.read_traffic(COUNTERS_MD, prec, nx, role_prefix + dom)
    out = dict(bound="hbm", kernel=dom, achieved=g, peak=PEAK_HBM / 1e9, unit="GB/s",
               frac=(g * 1e9 / PEAK_HBM) if g else None, traffic=traffic,
               method_bytes_per_launch=(g * 1e9 * avg_s) if g else None,
               share_of_step=kern[dom]["total_ms"] / (res["ms_per_step"] * res["steps"]),
               step_frac=res["value"] / step_roofline(res["S"]))
    if gd is not None:
        out["design_bytes_per_launch"] = gd * 1e9 * avg_s
        out["design_achieved"] = gd
        out["design_frac"] = gd * 1e9 / PEAK_HBM
    if traffic is not None:
        out["traffic_GBps"] = traffic / avg_s / 1e9
        if g:
            out["traffic_over_method_bytes"] = traffic / (g * 1e9 * avg_s)
    if rates:
        out["stream_read_GBps"] = rates["read"] / 1e9
        out["stream_copy_GBps"] = rates["copy"] / 1e9
        out["stream_write_GBps"] = rates["write"] / 1e9
        rw = design_rw(dom, 4, fused)
        if rw:
            ceil = stream_ceiling(rw[0], rw[1], rates["read"], rates["write"])
            out["design_reads_writes_S"] = list(rw)
            out["stream_ceiling_GBps"] = ceil / 1e9
            ach = gd if gd is not None else g
            out["frac_of_stream_ceiling"] = ach * 1e9 / ceil if ach else None
    return out


def cpu_baseline(nsample=1024, steps=3, workers=-1):
    """The FP64 oracle on a bounded sample of the same workload: nsample
    plane-wave states of the 32^3 trapped gas (trap + vortex), stationary
    start (one f evaluation), then `steps` AB4AM5 steps; the rate is
    nsample * steps / time of those steps.  workers: scipy.fft threads of
    the oracle (-1 = every host core, 1 = a single core)."""
    from oracle import lattice as L, bdg, functional as F, td
    from paper_2602_08982_amd import workloads as W
    import synth
    cfg = W.PLAIN
    lat = L.Lattice(*cfg["n"])
    kidx = W.all_kidx(cfg["n"])
    rng = synth.rng(5)
    sel = np.sort(rng.choice(len(kidx), size=nsample, replace=False))
    E, phi = bdg.plane_wave_states(lat, kidx[sel], cfg["u0"] - cfg["mu"], cfg["delta0"])
    dx, dy = synth.vortex_offset(2)
    phi = bdg.imprint_phase(phi, bdg.vortex_phase(lat, [(dx, dy, 1.0)]))
    vext = W.harmonic(cfg["n"], cfg["d"], cfg["omega"])
    lam = F.lambda_c(vext, cfg["mu"], 0.5 * np.pi ** 2)
    sysm = td.TDSystem(td.Geometry3D(lat), F.Functional(F.SLDA), cfg["mu"], vext, lam,
                       F.fermi_weight(E), F.fermi_weight(-E))
    saved = L._WORKERS
    L._WORKERS = workers
    try:
        p, hist, _ = td.start(sysm, phi, cfg["dt"], "AB4AM5", selfstart=0)
        t0 = time.perf_counter()
        for _ in range(steps):
            p, hist = td.abm_step(sysm, p, hist, cfg["dt"])
        dt = time.perf_counter() - t0
    finally:
        L._WORKERS = saved
    cores = os.cpu_count() if workers == -1 else workers
    return dict(value=nsample * steps / dt, unit="state-steps/s", cores=cores, kind="oracle",
                sample=f"{nsample} of the 32768 states of the 32^3 FP64 workload (seeded choice), "
                       f"{steps} AB4AM5 steps after a stationary start, timed steps only; "
                       f"scipy.fft with workers={workers} ({cores} host threads)", seconds=dt)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-q1d", action="store_true")
    ap.add_argument("--no-q2d", action="store_true")
    ap.add_argument("--aslda3d-steps", type=int, default=10,
                    help="steps of the spin-imbalanced (ASLDA) FP64 32^3 run, 32,768 states (0 = skip)")
    ap.add_argument("--q1d-aslda-steps", type=int, default=500,
                    help="steps of the spin-imbalanced (ASLDA) batched quasi-1D run (0 = skip)")
    ap.add_argument("--q2d-steps", type=int, default=100,
                    help="steps of the quasi-2D 64x64 (N_z = 64) workload, FP32-mixed; half as many in FP64")
    ap.add_argument("--no-warmstart", action="store_true")
    ap.add_argument("--warmstart-size", choices=["small", "medium", "default", "large"], default="default",
                    help="small: 8x8x4 lattice, 48 training / 8 held-out solves (seconds); medium: 16x16x8, "
                         "200 / 40 (about ten minutes); default: 24x24x8, 48 / 20, Broyden mixing only (about "
                         "four minutes); large: 24x24x8, 100 / 20, Broyden mixing only")
    ap.add_argument("--q1d-steps", type=int, default=2000,
                    help="steps of the batched quasi-1D run (one graph launch)")
    ap.add_argument("--q1d-fp64-steps", type=int, default=500,
                    help="steps of the FP64 run of the batched quasi-1D workload (one graph launch; 0 = skip)")
    ap.add_argument("--general-steps", type=int, default=None,
                    help="steps of the FP64 32^3 workload evolved with the general functional A = 1.094, after "
                         "the same warm-up (default: --steps, so that its cost compares with the A = 1 step; "
                         "0 = skip)")
    ap.add_argument("--q1d-eager", action="store_true",
                    help="run the batched quasi-1D steps eagerly (tdslda_abm_step) instead of one graph launch")
    ap.add_argument("--q1d-general-steps", type=int, default=500,
                    help="steps of the batched quasi-1D run with the general functional (A = 1.094; one graph "
                         "launch; 0 = skip)")
    ap.add_argument("--q1d-friction", action="store_true",
                    help="also time the batched quasi-1D run with the quantum-friction terms on")
    ap.add_argument("--mixed-steps", type=int, default=None,
                    help="steps of the FP32-mixed run and of its FP64 reference (default: --steps); the "
                         "errors of rho, nu and E are taken after them")
    ap.add_argument("--precision-track", type=int, default=0, metavar="STEPS",
                    help="also run the FP32-mixed 48^3 workload and its FP64 run for STEPS steps and report the "
                         "FP32-mixed errors of rho, nu and E every 50 steps (not timed)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a device-to-device copy of 4 GiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; the multi-GPU (state-sharded, "
              "density all-reduce) path is a design, not code here.", file=sys.stderr)
        sys.exit(2)
    if args.warmup < 1:
        args.warmup = 1
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calib:
        a = torch.ones(1 << 29, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_read_per_launch": a.numel() * 8,
                          "copy_calib_bytes_written_per_launch": b.numel() * 8, "launches": 3}))
        return
    from paper_2602_08982_amd import tdslda as T
    from paper_2602_08982_amd import workloads as W
    T.load_library()

    rates = stream_rates()
    plain = run_workload(W.PLAIN, args.steps, args.warmup, args.seed)
    plain["steps"] = args.steps
    print(f"# plain fp64 32^3: {plain['value']:.4g} state-steps/s, {plain['ms_per_step']:.2f} ms/step",
          file=sys.stderr, flush=True)
    plaingen = None
    gsteps = args.steps if args.general_steps is None else args.general_steps
    if gsteps > 0:
        plaingen = run_workload(W.PLAIN, gsteps, args.warmup, args.seed, A=1.094)
        plaingen["steps"] = gsteps
        print(f"# plain fp64 32^3, general functional A = 1.094: {plaingen['value']:.4g} state-steps/s, "
              f"{plaingen['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    mixed = None
    if not args.no_mixed:
        msteps = args.mixed_steps or args.steps
        mixed = run_workload(W.MIXED, msteps, args.warmup, 4, observe=True)
        mixed["steps"] = msteps
        print(f"# mixed fp32 48^3: {mixed['value']:.4g} state-steps/s, {mixed['ms_per_step']:.2f} ms/step",
              file=sys.stderr, flush=True)
        ref64 = run_workload(W.MIXED, msteps, args.warmup, 4, profile=False, precision=T.FP64,
                             observe=True)
        print(f"# fp64 48^3 (same states): {ref64['value']:.4g} state-steps/s, "
              f"{ref64['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
        o, r = mixed["obs"], ref64["obs"]
        mixed["vs_fp64"] = dict(
            fp64_value=ref64["value"], fp64_ms_per_step=ref64["ms_per_step"],
            speedup=mixed["value"] / ref64["value"],
            rho_rel_err=float(np.abs(o["rho"] - r["rho"]).max() / np.abs(r["rho"]).max()),
            nu_rel_err=float(np.abs(o["nu"] - r["nu"]).max() / np.abs(r["nu"]).max()),
            energy_rel_err=float(abs(o["energy"]["total"] - r["energy"]["total"]) / abs(r["energy"]["EFG"])))
    track = track_precision(args.precision_track, 50, args.warmup) if args.precision_track else None
    q1d_fric = None
    if args.q1d_friction:
        q1d_fric = run_q1d(args.q1d_steps, max(1, args.warmup), friction=True)
        print(f"# batched q1d with friction: {q1d_fric['value']:.4g} state-steps/s", file=sys.stderr, flush=True)
    q1d = None
    if not args.no_q1d:
        q1d = run_q1d(args.q1d_steps, max(1, args.warmup), eager=args.q1d_eager)
        print(f"# batched q1d: {q1d['value']:.4g} state-steps/s over {q1d['steps']} steps "
              f"({q1d['nst']} states), graph record {q1d['graph_record_ms']:.0f} ms", file=sys.stderr, flush=True)
    q1d64 = None
    if not args.no_q1d and args.q1d_fp64_steps > 0:
        q1d64 = run_q1d(args.q1d_fp64_steps, max(1, args.warmup), precision=T.FP64, profile_steps=0,
                        eager=args.q1d_eager)
        print(f"# batched q1d FP64: {q1d64['value']:.4g} state-steps/s over {q1d64['steps']} steps",
              file=sys.stderr, flush=True)
    q1dgen = None
    if not args.no_q1d and args.q1d_general_steps > 0:
        q1dgen = run_q1d(args.q1d_general_steps, max(1, args.warmup), A=1.094, eager=args.q1d_eager)
        print(f"# batched q1d, general functional A = 1.094: {q1dgen['value']:.4g} state-steps/s over "
              f"{q1dgen['steps']} steps", file=sys.stderr, flush=True)
    q1das = None
    if not args.no_q1d and args.q1d_aslda_steps > 0:
        q1das = run_q1d_aslda(args.q1d_aslda_steps, max(1, args.warmup))
        print(f"# batched q1d, spin-imbalanced ASLDA: {q1das['value']:.4g} state-steps/s over {q1das['steps']} "
              f"steps ({q1das['nst']} states, max polarisation {q1das['max_polarisation']:.2f})",
              file=sys.stderr, flush=True)
    as3 = None
    if args.aslda3d_steps > 0:
        as3 = run_aslda3d(args.aslda3d_steps, max(1, args.warmup))
        print(f"# FP64 32^3 spin-imbalanced ASLDA: {as3['value']:.4g} state-steps/s, {as3['ms_per_step']:.1f} "
              f"ms/step ({as3['nst']} states, max polarisation {as3['max_polarisation']:.2f})", file=sys.stderr,
              flush=True)
    q2d = q2d64 = None
    if not args.no_q2d and args.q2d_steps > 0:
        q2d = run_q2d(args.q2d_steps, max(1, args.warmup))
        print(f"# quasi-2D 64x64 (N_z = 64): {q2d['value']:.4g} state-steps/s, {q2d['ms_per_step']:.2f} ms/step "
              f"({q2d['nst']} states)", file=sys.stderr, flush=True)
        q2d64 = run_q2d(max(1, args.q2d_steps // 2), max(1, args.warmup), precision=T.FP64)
        print(f"# quasi-2D FP64: {q2d64['value']:.4g} state-steps/s, {q2d64['ms_per_step']:.2f} ms/step",
              file=sys.stderr, flush=True)
    warm = None
    if not args.no_warmstart:
        from paper_2602_08982_amd import warmstart as WS
        if args.warmstart_size == "small":
            wcfg, ntr, nte, ep = dict(WS.Q2D, nx=8, ny=8, nz=4, omega=0.48, channels=16, coarse=6), 48, 8, 200
        elif args.warmstart_size == "medium":
            wcfg, ntr, nte, ep = dict(WS.Q2D), 200, 40, 300
        else:
            ntr = 100 if args.warmstart_size == "large" else 48
            wcfg, nte, ep = dict(WS.Q2D, nx=24, ny=24, omega=0.16, coarse=18, linear=False), 20, 300
        warm = WS.experiment(wcfg, range(0, ntr), range(10000, 10000 + nte), epochs=ep,
                             log=lambda m: print("# warm start: " + m, file=sys.stderr, flush=True))
        if "warm_iters_mean" in warm:
            print(f"# warm start: {warm['warm_iters_mean']:.1f} vs plain {warm['plain_iters_mean']:.1f} iterations "
                  f"to r < 1e-8 ({warm['n_test']} held-out seeds)", file=sys.stderr, flush=True)
        if "warm_broyden_iters_mean" in warm:
            print(f"# Broyden mixing: warm {warm['warm_broyden_iters_mean']:.1f} vs plain "
                  f"{warm['plain_broyden_iters_mean']:.1f} iterations", file=sys.stderr, flush=True)
        if warm.get("symmetry_release_start"):
            rs = warm["symmetry_release_start"]
            for k in ("linear", "broyden"):
                if k in rs:
                    print(f"# symmetry-release start ({k} mixing): {rs[k]['q1d_iters']} quasi-1D + "
                          f"{rs[k]['q2d_iters_mean']:.1f} quasi-2D iterations = {rs[k]['target_equivalent']:.1f} "
                          f"target-equivalent (cost ratio {rs['cost_ratio']:.4f})", file=sys.stderr, flush=True)
        if warm.get("coarse_start"):
            cs = warm["coarse_start"]
            for k in ("linear", "broyden"):
                if k in cs:
                    print(f"# coarse-lattice start ({k} mixing): {cs[k]['coarse_iters_mean']:.1f} coarse + "
                          f"{cs[k]['fine_iters_mean']:.1f} target iterations = {cs[k]['target_equivalent']:.1f} "
                          f"target-equivalent (cost ratio {cs['cost_ratio']:.3f})", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline()
        cpu["single_core"] = cpu_baseline(nsample=128, steps=2, workers=1)
        print(f"# cpu oracle: {cpu['value']:.4g} state-steps/s ({cpu['cores']} threads), "
              f"{cpu['single_core']['value']:.4g} on one core", file=sys.stderr, flush=True)

    line = {
        "metric": "TDSLDA quasiparticle state-steps/s + %HBM roofline, FP32-mixed vs FP64",
        "value": plain["value"],
        "unit": "state-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": plain["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "plain FP64 32^3 trapped gas, one vortex (AB4AM5, dt=0.005)",
                   "lattice": [32, 32, 32], "states_evolved": plain["nst"],
                   "states_represented": 2 * plain["nst"], "integrator": "AB4AM5"},
        "roofline": roofline(plain, rates, "double", 32),
        "cpu_baseline": cpu,
        "kernels": plain["kernels"],
        "check": plain["check"],
    }
    if plaingen is not None:
        pk = plaingen["kernels"]
        line["general_functional_3d"] = {
            "workload": "the FP64 32^3 workload (same start) evolved with the general functional A = 1.094 "
                        "(alpha = A, current potential (1 - A) j / rho; Eq. h_sigma with Eq. kinop-alpha: line "
                        "passes per axis, 7 transforms per component and axis)",
            "value": plaingen["value"], "unit": "state-steps/s", "ms_per_step": plaingen["ms_per_step"],
            "steps": plaingen["steps"],
            "cost_vs_A1": plaingen["ms_per_step"] / plain["ms_per_step"],
            "cost_vs_A1_note": "same steps and warm-up as the A = 1 run (one predictor pass and one closing F-only "
                               "evaluation per call in both)",
            "kernels": {k: dict(launches=v["launches"], avg_ms=v["avg_ms"]) for k, v in pk.items()},
            "check": plaingen["check"],
        }
    if mixed is not None:
        line["fp32_mixed"] = {
            "workload": "FP32-mixed 48^3 elongated trap, vortex pair, 8192 lowest-|E| states",
            "value": mixed["value"], "unit": "state-steps/s", "ms_per_step": mixed["ms_per_step"],
            "steps": mixed["steps"],
            "dtype": "f32 states / f64 sums", "roofline": roofline(mixed, rates, "float", 48), "kernels": mixed["kernels"],
            "check": mixed["check"], "vs_fp64_same_workload": mixed["vs_fp64"],
        }
    if track is not None:
        line["fp32_mixed_error_track"] = track
    if q1d_fric is not None:
        line["batched_q1d_friction"] = {
            "workload": "the batched quasi-1D run with the quantum-friction terms on (alpha = beta = 5, gamma = 0.1)",
            "value": q1d_fric["value"], "unit": "state-steps/s", "ms_per_step": q1d_fric["ms_per_step"],
            "kernels": q1d_fric["kernels"], "check": q1d_fric["check"],
        }
    if q1d is not None:
        line["batched_q1d"] = {
            "workload": "2,304 quasi-1D problems (48x48 k_perp), N_z=256, |E|<12, FP32 states / FP64 sums, "
                        f"{q1d['steps']} AB4AM5 steps " + ("eagerly" if args.q1d_eager else "in one HIP-graph launch"),
            "value": q1d["value"], "unit": "state-steps/s", "ms_per_step": q1d["ms_per_step"],
            "states_evolved": q1d["nst"], "graph_record_ms": q1d["graph_record_ms"],
            "setup_seconds": q1d["setup_seconds"], "tuned_workgroups": q1d["tuned"],
            "problems": q1d["problems"], "kernels": q1d["kernels"], "check": q1d["check"],
            "roofline": roofline(dict(q1d, steps=q1d["profile_steps"]), rates, "float", 16, "q1d_", fused=True)
            if q1d["kernels"] else None,
        }
        if q1d64 is not None:
            line["batched_q1d"]["vs_fp64_same_workload"] = dict(
                fp64_value=q1d64["value"], fp64_ms_per_step=q1d64["ms_per_step"], fp64_steps=q1d64["steps"],
                speedup=q1d["value"] / q1d64["value"], fp64_check=q1d64["check"])
    if q1dgen is not None:
        line["batched_q1d_general_functional"] = {
            "workload": "the batched quasi-1D workload (same initial states) evolved with the general functional "
                        "A = 1.094 (alpha = A, current potential (1 - A) j / rho; Eq. h_sigma with Eq. "
                        f"kinop-alpha, 7 transforms per component), {q1dgen['steps']} steps "
                        + ("eagerly" if args.q1d_eager else "in one HIP-graph launch"),
            "value": q1dgen["value"], "unit": "state-steps/s", "ms_per_step": q1dgen["ms_per_step"],
            "cost_vs_A1": (q1dgen["ms_per_step"] / q1d["ms_per_step"]) if q1d else None,
            "kernels": q1dgen["kernels"], "check": q1dgen["check"],
            "roofline": roofline(dict(q1dgen, steps=q1dgen["profile_steps"]), rates, "float", 16, "q1dgen_",
                                 fused=True) if q1dgen["kernels"] else None,
        }
    if q1das is not None:
        line["batched_q1d_aslda"] = {
            "workload": "spin-imbalanced ASLDA (p != 0), 576 quasi-1D problems (24x24 k_perp), N_z = 64, "
                        "mu_a = 1.3, mu_b = 0.5, both branches with |E| < 6 from the device eigensolver, FP32 "
                        f"states / FP64 sums, {q1das['steps']} AB4AM5 steps in one HIP-graph launch",
            "value": q1das["value"], "unit": "state-steps/s", "ms_per_step": q1das["ms_per_step"],
            "states_evolved": q1das["nst"], "max_polarisation": q1das["max_polarisation"],
            "setup_seconds": q1das["setup_seconds"], "tuned_workgroups": q1das["tuned"],
            "kernels": q1das["kernels"], "check": q1das["check"], "problems": q1das["problems"],
        }
    if as3 is not None:
        line["aslda_3d"] = {
            "workload": "spin-imbalanced ASLDA (p != 0), FP64 32^3 trap (omega = 0.05), mu_a = 1.4, mu_b = 0.6, "
                        "both branches of the 16,384 lowest-|xi| momenta of the uniform start (32,768 states), "
                        f"{as3['steps']} AB4AM5 steps (the general line passes with per-spin fields)",
            "value": as3["value"], "unit": "state-steps/s", "ms_per_step": as3["ms_per_step"],
            "states_evolved": as3["nst"], "max_polarisation": as3["max_polarisation"],
            "cost_per_state_vs_A1": (as3["ms_per_step"] / as3["nst"]) / (plain["ms_per_step"] / plain["nst"]),
            "setup_seconds": as3["setup_seconds"], "kernels": as3["kernels"], "check": as3["check"],
        }
    if q2d is not None:
        line["quasi2d"] = {
            "workload": "quasi-2D trapped gas, 64x64 x-y lattice, N_z = 64 plane waves along z (33 |k_z| "
                        "classes), one vortex line, all 135,168 plane-wave states, FP32 states / FP64 sums, "
                        f"{q2d['steps']} AB4AM5 steps (one launch per kernel)",
            "value": q2d["value"], "unit": "state-steps/s", "ms_per_step": q2d["ms_per_step"],
            "states_evolved": q2d["nst"], "setup_seconds": q2d["setup_seconds"], "kernels": q2d["kernels"],
            "check": q2d["check"],
            "roofline": roofline(dict(q2d, steps=q2d["profile_steps"]), rates, "float", 64, "q2d_", fused=True)
            if q2d["kernels"] else None,
            "fp64": dict(value=q2d64["value"], ms_per_step=q2d64["ms_per_step"], steps=q2d64["steps"],
                         kernels=q2d64["kernels"], check=q2d64["check"],
                         roofline=roofline(dict(q2d64, steps=q2d64["profile_steps"]), rates, "double", 64, "q2d_",
                                           fused=True) if q2d64["kernels"] else None),
        }
    if warm is not None:
        line["learned_warm_start"] = {
            "workload": f"static quasi-2D solve, {warm['lattice'][0]}x{warm['lattice'][1]} x-y lattice, "
                        f"{warm['lattice'][2]} k_z modes, trap + 1-4 obstacles, fixed N, linear mixing 0.5 "
                        f"(and modified Broyden mixing, history {warm.get('broyden', 0)})",
            "metric": "mixing iterations to r < 1e-8, mean over held-out seeds",
            "warm": warm.get("warm_iters_mean"), "plain": warm.get("plain_iters_mean"), "fallbacks": warm["fallbacks"],
            "warm_broyden": warm.get("warm_broyden_iters_mean"), "plain_broyden": warm.get("plain_broyden_iters_mean"),
            "n_train": warm["n_train"], "n_test": warm["n_test"],
            "seconds_per_iteration": warm["seconds_per_iteration"],
            "train_data_seconds": warm["train_data_seconds"], "fit_seconds": warm["fit_seconds"],
            "coarse_lattice_start": warm.get("coarse_start"),
            "symmetry_release_start": warm.get("symmetry_release_start"),
        }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
