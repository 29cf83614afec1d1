"""Benchmark of the DG thermosphere hot path on one MI355X.

Default workload: the cubed-sphere shell 6 x 16 x 16 angular x 16 radial elements
(stretch 1.15), p = 3, 5 fields: 24,576 elements, 7,864,320 DOF. A step is one
evaluation of the residual R(u) (the operator every Newton, GMRES and DIRK stage
is built from); J(u)v in FP64 and FP32 is timed the same way and reported beside
it, and so are the implicit DIRK(3,3) step on the same shell (FP64 and FP32 J v)
and the batch of 4096 radial columns advanced 100 steps in one launch. Inputs are
resident in HBM before the timed regions. Prints one JSON line.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload shell-p3|shell-p4]
                    [--only residual] [--mode warmstart]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name, seed=0):
    import synth
    if name == "shell-p3":
        return synth.config_shell_p3(seed)
    if name == "shell-p4":
        return synth.config_shell_p4(seed)
    raise SystemExit("unknown workload %s" % name)


def shell_state(w, X):
    """state at the library's nodes X [E, N, 3]"""
    import synth
    return synth.shell_state_at(w, X)


def pass1_bytes(w, prec_bytes=8):
    """algorithmic HBM bytes of one launch of the element pass (pass 1): read the
    state (plus the tangent for J v), write the partial residual, write the face
    traces F.Sn of all 6 faces, read the angular tables once per angular cell"""
    n = w.p + 1
    N, N2 = n ** 3, n ** 2
    E = w.n_elem
    A = 6 * w.n_ang ** 2
    per_elem = 5 * N * 8 + 5 * N * prec_bytes + 6 * 5 * N2 * prec_bytes
    return E * per_elem + A * 13 * N2 * 8


def pass1_flops(p):
    """algorithmic FP64 operations of the element pass per node (an FMA counts 2, an
    exp, log, sqrt or division 1), n = p + 1 nodes per direction, phi = 6/n face slots
    per node:
      line coefficients 16n; gradient 5(14n + 9); lift 30 phi; pointwise flux and
      source 246, heating 18, node geometry 20; contravariant fluxes 75; divergence
      5(6n + 2); face slots (trace 10, sigma and Z on the owned half 45/2, own half and
      sent trace 35) 67.5 phi"""
    n = p + 1
    phi = 6.0 / n
    return 16 * n + 5 * (14 * n + 9) + 30 * phi + 246 + 18 + 20 + 75 + 5 * (6 * n + 2) + 67.5 * phi


# HBM counter scale factors measured on MI355X with a 256 MiB device copy (rocprofv3
# --pmc FETCH_SIZE / WRITE_SIZE): FETCH_SIZE reads half the bytes a kernel fetches,
# WRITE_SIZE the bytes it writes
FETCH_SCALE = 2.0
WRITE_SCALE = 1.0


def pass2_bytes(w):
    """algorithmic HBM bytes of the trace pass (pass 2): read the 6 x 5 x (p+1)^2 incoming
    trace slots of every element, read and write R on its face nodes"""
    n = w.p + 1
    N, N2 = n ** 3, n ** 2
    Nface = N - (n - 2) ** 3
    return w.n_elem * (6 * 5 * N2 * 8 + 2 * 5 * Nface * 8)


def residual_bytes(w):
    """algorithmic HBM bytes of one full R(u) as this design moves them (both passes)"""
    return pass1_bytes(w) + pass2_bytes(w)


# reference roofline of R(u): a two-pass LDG evaluation with a stored gradient moves
# 8 (3 + 2d) = 72 bytes per DOF in 3D (pass 1 reads u and writes q, pass 2 reads u and q and
# writes R); the target is half of that roofline
R_REF_BYTES_PER_DOF = 72.0
HBM_TARGET_FRAC = 0.5
FP64_RIDGE = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)     # flop per byte


def element_pass_roofline(fl1, b1, p1_ms, tr_bytes, tr_detail, counters):
    """the element pass against the roof its arithmetic intensity selects: below the FP64
    ridge (78.6 TFLOP/s / 8 TB/s = 9.8 flop/B) that is HBM, above it the FP64 vector peak.
    Both fractions are reported, with the VALU issue fraction from the counters where a
    counter run of this kernel exists"""
    ai = fl1 / b1
    gbs = b1 / (p1_ms * 1e-3) / 1e9
    tflops = fl1 / (p1_ms * 1e-3) / 1e12
    bound = "hbm" if ai < FP64_RIDGE else "alu"
    out = {"bound": bound,
           "achieved": gbs if bound == "hbm" else tflops,
           "peak": HBM_PEAK_GBS if bound == "hbm" else FP64_PEAK_TFLOPS,
           "unit": "GB/s" if bound == "hbm" else "TFLOP/s",
           "frac": gbs / HBM_PEAK_GBS if bound == "hbm" else tflops / FP64_PEAK_TFLOPS,
           "traffic": tr_bytes, "traffic_detail": tr_detail,
           "kernel": "shell_pass1 (R, f64)",
           "arithmetic_intensity_flop_per_byte": ai, "fp64_ridge_flop_per_byte": FP64_RIDGE,
           "algorithmic_bytes_per_launch": b1, "algorithmic_flops_per_launch": fl1,
           "avg_launch_ms": p1_ms, "hbm_gbs_algorithmic": gbs, "hbm_frac_algorithmic": gbs / HBM_PEAK_GBS,
           "fp64_tflops_algorithmic": tflops, "fp64_frac_algorithmic": tflops / FP64_PEAK_TFLOPS}
    if tr_bytes:
        out["hbm_frac_counters"] = tr_bytes / (p1_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
        out["traffic_over_algorithmic"] = tr_bytes / b1
    if counters:
        out.update(counters)
    return out


# HBM bytes per launch of the element pass (FP64 R) from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs of `bench.py --only residual --copy-probe`, scaled as above, keyed by
# workload and launch configuration, with the hash of the kernel sources they were taken
# on (a changed kernel reports null until measured again)
PASS1_PROFILE = "profiles/shell_pass1_shell_pass2_R_shell-p3-7.9M_all-configs_counters.txt"
PASS1_TRAFFIC = {
    ("shell-p3", 0): {"src": "ac03b2dda95fd231", "fetch_kib": 50360.8, "write_kib": 151680.0, "valu_insts": 4.4062e+07,
                      "profile": PASS1_PROFILE},
    ("shell-p3", 1): {"src": "ac03b2dda95fd231", "fetch_kib": 49949.3, "write_kib": 151680.0, "valu_insts": 4.3471e+07,
                      "profile": PASS1_PROFILE},
    ("shell-p3", 2): {"src": "ac03b2dda95fd231", "fetch_kib": 50356.4, "write_kib": 151680.0, "valu_insts": 4.4062e+07,
                      "profile": PASS1_PROFILE},
    ("shell-p3", 3): {"src": "ac03b2dda95fd231", "fetch_kib": 49854.1, "write_kib": 151680.0, "valu_insts": 4.3183e+07,
                      "profile": PASS1_PROFILE},
    ("shell-p3", 4): {"src": "ac03b2dda95fd231", "fetch_kib": 49824.7, "write_kib": 151680.0, "valu_insts": 4.3677e+07,
                      "profile": PASS1_PROFILE},
    ("shell-p3", 5): {"src": "ac03b2dda95fd231", "fetch_kib": 175558.5, "write_kib": 309593.5, "valu_insts": 4.3331e+07,
                      "profile": PASS1_PROFILE},
}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    # the files the FP64 residual's element pass is built from (shell_r64.hip instantiates it)
    for f in ("paper_2306_01085_amd/csrc/shell_pass1.h", "paper_2306_01085_amd/csrc/shell_r64.hip",
              "paper_2306_01085_amd/csrc/dg_common.h", "paper_2306_01085_amd/csrc/internal.h"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    import __graft_entry__   # the element kernels' compiler flags change their code as well
    fl = __graft_entry__.FLAGS + __graft_entry__.PER_SOURCE.get("shell_r64.hip", [])
    fl = [f for i, f in enumerate(fl) if f != "-I" and (i == 0 or fl[i - 1] != "-I")]   # not the paths
    h.update(" ".join(fl).encode())
    return h.hexdigest()[:16]


def traffic(workload, cfg):
    """(HBM bytes per launch, detail) or (None, reason)"""
    t = PASS1_TRAFFIC.get((workload, cfg))
    if t is None:
        return None, "no counter run for this workload and configuration"
    if t["src"] != kernel_source_hash():
        return None, "kernel changed since the counters were taken"
    fetch = t["fetch_kib"] * 1024 * FETCH_SCALE
    write = t["write_kib"] * 1024 * WRITE_SCALE
    return fetch + write, {"fetch_bytes": fetch, "write_bytes": write, "profile": t["profile"]}


# VALU issue: a wave64 VALU instruction occupies a SIMD (16 lanes) for 4 cycles; 1024 SIMDs
CHIP_SIMDS = 1024
CLOCK_GHZ = 2.4


def valu_counters(workload, cfg, p1_ms):
    """VALU issue fraction of the element pass at the measured launch time, from the
    SQ_INSTS_VALU count of its counter run (None if the kernel changed since)"""
    t = PASS1_TRAFFIC.get((workload, cfg))
    if t is None or "valu_insts" not in t or t["src"] != kernel_source_hash():
        return {}
    cycles = p1_ms * 1e-3 * CLOCK_GHZ * 1e9
    return {"valu_insts_per_launch": t["valu_insts"],
            "valu_issue_frac": t["valu_insts"] * 4.0 / (CHIP_SIMDS * cycles),
            "valu_note": "SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x launch time x 2.4 GHz)"}


def _cpu_info():
    """model name and socket count of the host, and the threads this process may use"""
    model, sockets = None, set()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                k = k.strip()
                if k == "model name" and model is None:
                    model = v.strip()
                elif k == "physical id":
                    sockets.add(v.strip())
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "sockets": len(sockets) or None, "os_cpu_count": os.cpu_count(), "usable_threads": usable}


def _median_time(fn, budget_s, max_runs, warm=True):
    if warm:
        fn()
    times = []
    t_end = time.perf_counter() + budget_s
    while len(times) < max_runs and (len(times) < min(2, max_runs) or time.perf_counter() < t_end):
        t0 = time.perf_counter()
        fn()
        times.append(time.perf_counter() - t0)
    return float(np.median(times)), len(times)


def cpu_baseline(w, implicit=None, budget_s=4.0):
    """the FP64 oracle timed on this host's cores, on bounded samples of the workloads:
    R(u) and the complex-step J(u)v on a shell of 6 x 8 x 8 x 16 elements at the benchmark's
    degree (a quarter of the benchmark shell) with one BLAS thread and with every usable
    thread; one dense-Newton implicit DIRK(3,3) step of the 64-element p = 2 column (dt = 10 s)
    with one thread; and the implicit steps of the shells extrapolated from the R and J v
    counts of the GPU's FP64 runs times the oracle's per-call time scaled by DOF (labelled
    as extrapolations: they leave out the preconditioner and the Krylov vector work, a
    lower bound). `value` is the one-thread R(u) rate."""
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import dg as odg
    from oracle import jac as ojac
    from oracle import mesh as omesh
    from oracle import timeint
    info = _cpu_info()
    n_ang, n_rad = 8, w.n_rad
    om = omesh.shell_mesh(w.p, n_ang, n_rad, w.r_bot, w.r_top, w.stretch)
    u = np.moveaxis(w.state_fn()(om.X), 0, 1).copy()
    v = synth.tangent(u.shape, 1)
    ndof = u.size
    res = {}
    for label, threads in (("1_thread", 1), ("all_threads", info["usable_threads"])):
        with threadpool_limits(limits=threads):
            tr, nr = _median_time(lambda: odg.residual(om, w.phys, u, 0.0), budget_s, 15)
            tj, nj = _median_time(lambda: ojac.jvp_complex(om, w.phys, u, v, 0.0), budget_s, 10)
        res[label] = {"threads": threads, "residual_s": tr, "residual_gdofs": ndof / tr / 1e9, "residual_runs": nr,
                      "jvp_s": tj, "jvp_gdofs": ndof / tj / 1e9, "jvp_runs": nj}
    # one implicit step of the 1D column workload (64 elements, p = 2, 576 DOF), dense Newton
    wc = synth.config_column(0)
    cm = omesh.columns_mesh([int(wc.nelem[0])], int(wc.p[0]), wc.r_bot, wc.r_top)
    Pc = dict(wc.phys)
    for k in wc.col_phys:
        Pc[k] = float(wc.col_phys[k][0])
    uc = np.moveaxis(wc.state(0, cm.X[:, :, 0]), 0, 1).copy()
    with threadpool_limits(limits=1):
        tc, ncr = _median_time(lambda: timeint.implicit_step_dense(cm, Pc, uc, 0.0, wc.dt, scheme=33, rtol=1e-8),
                               0.0, 1, warm=False)
    out = {"value": res["1_thread"]["residual_gdofs"], "unit": "GDOF/s", "cores": 1, "kind": "oracle",
           "sample": "R(u) of the oracle on a 6x%dx%dx%d p=%d shell (%d DOF), median of %d runs, 1 BLAS thread"
                     % (n_ang, n_ang, n_rad, w.p, ndof, res["1_thread"]["residual_runs"]),
           "cpu": info, "shell_sample": res,
           "column_implicit_step": {"workload": "column-64-p2 (576 DOF), dt 10 s, DIRK(3,3), dense Newton 1e-8",
                                    "s_per_step": tc, "runs": ncr, "threads": 1},
           "note": "the oracle is a plain NumPy correctness reference, not a tuned CPU solver"}
    if implicit:
        per_dof = {k: res["1_thread"][k + "_s"] / ndof for k in ("residual", "jvp")}
        ext = {}
        for key, (n_dof, counts) in implicit.items():
            n_r = counts["newton_per_step"] + 3           # a residual per Newton iteration and per stage end
            n_j = counts["gmres_per_step"]
            ext[key] = {"n_dof": n_dof, "residuals_per_step": n_r, "jvps_per_step": n_j,
                        "s_per_step_extrapolated": n_dof * (n_r * per_dof["residual"] + n_j * per_dof["jvp"]),
                        "kind": "extrapolation (1 thread, lower bound)"}
        out["implicit_step_extrapolated"] = ext
    return out


FILTER_RATE = 0.5   # modal filter after every implicit step (per unit nondimensional time)
LINE_PC_EVERY = 16       # the radial-line preconditioner is rebuilt every 16 steps (at dt = 60 s the
                         # GMRES counts of 16 steps are those of a rebuild every 4 or 8 steps)
LINE_PC_PRECISION = 16   # and its factors are read as bf16 (same GMRES counts as double here)


def copy_probe(dev):
    """one plain device copy of 256 MiB: its FETCH_SIZE / WRITE_SIZE readings calibrate
    the HBM counters of the same run"""
    import torch
    src = torch.empty(2 ** 28 // 8, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()


def network_rates(w, steps, warmup, timed):
    """the warm-start network at its per-stage size (one row per element of the shell,
    15 (p+1)^3 inputs -> 128 -> 128 -> 5 (p+1)^3 outputs): inference (BF16 MFMA, FP32
    accumulation) against the dense BF16 peak, and one training step (FP32 backward and
    Adam) against the FP32 vector peak; algorithmic flops 2 x parameters per row forward,
    6 x per row for forward + backward"""
    import torch

    from paper_2306_01085_amd import Network
    from paper_2306_01085_amd import warmstart as wsm
    nin, nout = 15 * (w.p + 1) ** 3, 5 * (w.p + 1) ** 3
    if nin % 8 or nout % 32:
        return {"skipped": "the network's layer widths (%d in, %d out) are not multiples of 8 and 32 at p = %d"
                           % (nin, nout, w.p)}
    net = Network(nin, nout, wsm.init_params(np.random.default_rng(0), nin, nout))
    rows = w.n_elem
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn(rows, nin, device="cuda", generator=g)
    y = torch.empty(rows, nout, device="cuda")
    tgt = torch.randn(rows, nout, device="cuda", generator=g)
    f_inf = lambda: net.forward(x, out=y)
    f_trn = lambda: (net.grad(x, tgt, want_loss=False), net.adam_step(1e-4))
    for _ in range(warmup):
        f_inf()
    ms_inf = timed(f_inf, steps)
    f_trn()
    ms_trn = timed(f_trn, max(3, steps // 4))
    flops = 2.0 * net.n_params * rows
    out = {"rows": rows, "parameters": int(net.n_params), "inference_ms": ms_inf,
           "inference_tflops": flops / (ms_inf * 1e-3) / 1e12, "inference_peak_tflops": BF16_PEAK_TFLOPS,
           "train_step_ms": ms_trn, "train_step_tflops": 3 * flops / (ms_trn * 1e-3) / 1e12,
           "train_peak_tflops": FP32_PEAK_TFLOPS}
    del net, x, y, tgt
    torch.cuda.empty_cache()
    return out


def implicit_steps(w, mesh, u, n_steps, only=None):
    """seconds per DIRK(3,3) step of dt = 60 s at a 1e-8 relative Newton tolerance,
    GMRES(30) right-preconditioned by the radial-line block-Jacobi preconditioner,
    (rebuilt every LINE_PC_EVERY steps, bf16 factors), Eisenstat-Walker GMRES tolerances,
    plain extrapolated guess: FP64 vs FP32 vs BF16 J v, and the FP64 finite difference of R
    that section 3.2 describes; plus the FP32 run without a
    preconditioner and the FP32 run with the reduced basis of the 4 latest Newton updates
    on top of the line preconditioner"""
    import torch

    from paper_2306_01085_amd import DgError
    res = {"dt_s": 60.0, "newton_rtol": 1e-8,
           "gmres": "GMRES(30), CGS2, radial-line block-Jacobi preconditioner, Eisenstat-Walker tolerances",
           "steps": n_steps, "filter_rate": FILTER_RATE}
    runs = [(prec, 2, prec, 0) for prec in ("f64", "f32") + (("bf16",) if w.p in (3, 4) else ())]
    runs.append(("f64_fd", 2, "f64_fd", 0))   # the paper's finite-difference J v (section 3.2)
    runs.append(("f32_rb4", 2, "f32", 4))   # plus the reduced basis of the 4 latest Newton updates
    runs.append(("f32_no_precond", 0, "f32", 0))
    if only:
        runs = [r for r in runs if r[0] in only]
    mesh.set_option("line_pc_every", LINE_PC_EVERY)
    mesh.set_option("line_pc_precision", LINE_PC_PRECISION)
    res["line_pc_every"] = LINE_PC_EVERY
    res["line_pc_precision"] = LINE_PC_PRECISION
    for key, pc, prec, n_rb in runs:
        x = u.clone()
        t = 0.0
        secs, newton, gmres = [], [], []
        failed = None
        for _ in range(n_steps):
            try:
                st = mesh.implicit_step(x, t, w.dt, jvp_prec=prec, precond=pc, max_newton=15, max_restarts=40,
                                        filter_rate=FILTER_RATE, forcing=1, n_rb=n_rb)
            except DgError as ex:
                failed = str(ex)
                log("  implicit step (%s) failed: %s" % (key, failed))
                break
            t += w.dt
            secs.append(st["seconds"])
            newton.append(sum(st["newton_its"]))
            gmres.append(sum(st["gmres_its"]))
            log("  implicit step (%s): %.3f s, Newton %s, GMRES %s" % (key, st["seconds"], st["newton_its"],
                                                                   st["gmres_its"]))
        res[key] = {"s_per_step": float(np.mean(secs)) if secs else None,
                    "newton_per_step": float(np.mean(newton)) if newton else None,
                    "gmres_per_step": float(np.mean(gmres)) if gmres else None, "failed": failed}
        del x
        torch.cuda.empty_cache()
    return res


def implicit_steps_shell(name, n_steps, runs):
    """the implicit steps on another shell workload (its own mesh and state)"""
    import torch

    from paper_2306_01085_amd import Mesh
    w = workload(name)
    mesh = Mesh.shell(p=w.p, n_ang=w.n_ang, n_rad=w.n_rad, r_bot=w.r_bot, r_top=w.r_top, stretch=w.stretch,
                      phys=w.phys)
    u = torch.from_numpy(shell_state(w, mesh.nodes().reshape(w.n_elem, -1, 3)).ravel()).cuda()
    res = implicit_steps(w, mesh, u, n_steps, only=runs)
    res["workload"] = w.name
    res["n_dof"] = w.n_dof
    del mesh, u
    torch.cuda.empty_cache()
    return res


def column_batch(n_steps=None):
    """the batched radial-column sweep: 4096 columns advanced n_steps DIRK(3,3) steps of
    10 s in one persistent launch (autotuned grid), columns/s, in two discretisations: the
    over-integrated residual without a filter (the paper's weak form) and the collocated one
    with the modal filter. Also one step of the whole batch from the same start, kept for
    sampled columns (the smallest column of each degree) that the CPU-baseline leg compares
    with the oracle. Returns (report, samples)."""
    import torch

    import synth
    from paper_2306_01085_amd import Mesh
    from paper_2306_01085_amd import autotune
    w = synth.column_batch_workload(0)
    n_steps = n_steps or w.n_steps
    gm = Mesh.columns(w.nelem, w.p, w.r_bot, w.r_top, w.stretch, w.phys, w.col_phys)
    r = gm.nodes()
    off = gm.col_offsets()
    u0 = np.empty(gm.n_dof)
    for c in range(gm.n_col):
        rc = r[off[c] // 3:off[c + 1] // 3].reshape(w.nelem[c], w.p[c] + 1)
        u0[off[c]:off[c + 1]] = np.moveaxis(w.state(c, rc), 0, 1).ravel()
    u = torch.from_numpy(u0).cuda()
    pick = [int(np.flatnonzero(w.p == p)[np.argmin(w.nelem[w.p == p])]) for p in (2, 3, 4)]
    report, samples = {}, {"workload": w, "u0": u0, "offsets": off, "columns": pick, "runs": {}}
    for name, quad, rate in (("over_integrated", 1, 0.0), ("collocated_filtered", 0, FILTER_RATE)):
        gm.set_option("column_quadrature", quad)
        # trials of 32 steps: every call starts with a Jacobian build for every column, which
        # shorter trials overweight (they favour small grids, whose builds thrash the caches less)
        grid, _ = autotune.tune_columns(gm, u, 0.0, w.dt, steps=32, tag="q%d" % quad, log=log)
        policy, _ = autotune.tune_columns_policy(gm, u, 0.0, w.dt, steps=32, tag="q%d" % quad, log=log)
        x = u.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, st = gm.columns_integrate(x, 0.0, w.dt, n_steps, filter_rate=rate, raise_on_failure=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = np.asarray(st)
        report[name] = {"quadrature": "p + 2 Gauss points, exact mass matrix" if quad else "GLL collocation",
                        "filter_rate": rate, "seconds": el, "columns_per_s": gm.n_col / el, "grid": grid,
                        "chord_rebuild": {"slow_pct": policy[0], "stale_its": policy[1], "every_steps": 32},
                        "newton_per_step_mean": float(np.asarray(its).mean() / n_steps),
                        "failed": int((st != 0).sum()),
                        "failed_columns": [{"column": int(c), "elements": int(w.nelem[c]), "p": int(w.p[c]),
                                            "T_inf_K": float(w.T_inf[c]), "status": int(st[c])}
                                           for c in np.flatnonzero(st)[:8]]}
        x = u.clone()
        gm.columns_integrate(x, 0.0, w.dt, 1, filter_rate=rate, raise_on_failure=False)
        y = x.cpu().numpy()
        samples["runs"][name] = {"quad": quad, "rate": rate,
                                 "states": {c: y[off[c]:off[c + 1]].copy() for c in pick}}
    out = {"n_col": gm.n_col, "n_dof": gm.n_dof, "steps": n_steps, "newton_rtol": 1e-8}
    out.update(report)
    # the headline rate: the paper's discretisation (no filter)
    out["columns_per_s"] = report["over_integrated"]["columns_per_s"]
    out["failed"] = report["over_integrated"]["failed"]
    return out, samples


def column_sample_error(samples):
    """(CPU-baseline leg) the oracle's dense-Newton DIRK(3,3) step of the sampled batch
    columns in each discretisation, timed, and the GPU batch's step against it: relative
    error |u_gpu - u_oracle| / |u_oracle - u_0| per column"""
    from threadpoolctl import threadpool_limits

    from oracle import dg as odg
    from oracle import mesh as omesh
    from oracle import timeint
    w = samples["workload"]
    off = samples["offsets"]
    out = {}
    for name, run in samples["runs"].items():
        rows = []
        for c in samples["columns"]:
            om = omesh.columns_mesh([int(w.nelem[c])], int(w.p[c]), w.r_bot, w.r_top, float(w.stretch[c]))
            P = dict(w.phys)
            for k in w.col_phys:
                P[k] = float(w.col_phys[k][c])
            start = samples["u0"][off[c]:off[c + 1]].reshape(-1, 3, w.p[c] + 1).copy()
            t0 = time.perf_counter()
            with threadpool_limits(limits=1):
                ref, _ = timeint.implicit_step_dense(om, P, start, 0.0, w.dt, rtol=1e-9, filter_rate=run["rate"],
                                                     residual=odg.residual_overint if run["quad"] else None)
            tc = time.perf_counter() - t0
            got = run["states"][c].reshape(ref.shape)
            rows.append({"column": int(c), "elements": int(w.nelem[c]), "p": int(w.p[c]), "dof": int(got.size),
                         "rel_err_vs_oracle": float(np.linalg.norm(got - ref) / np.linalg.norm(ref - start)),
                         "oracle_s_per_step": tc})
        out[name] = rows
    return out


def warmstart_experiment(w, mesh, u, train_steps=60, eval_steps=8, every=4, epochs=8, eval_seed=None):
    """train the warm-start network on stages the method generates from the shell state
    (dt = 60 s, FP64 J v), then run eval_steps steps twice from the same state, plain and
    learned, with FP64 and with FP32 J v: by default the steps that follow the training
    trajectory; with eval_seed, a held-out trajectory from t = 0 of the workload drawn with
    that seed (another temperature profile, perturbation and heating peak)"""
    import torch

    from paper_2306_01085_amd import Network
    from paper_2306_01085_amd import warmstart as wsm
    opts = dict(newton_rtol=1e-8, precond=2, max_newton=30, max_restarts=40, filter_rate=FILTER_RATE, forcing=1)
    # a fresh preconditioner every step, so that the plain and learned runs see the same one
    mesh.set_option("line_pc_every", 1)
    mesh.set_option("line_pc_precision", LINE_PC_PRECISION)
    nin, nout = 15 * (w.p + 1) ** 3, 5 * (w.p + 1) ** 3
    cap = (3 * train_steps) * ((w.n_elem + every - 1) // every)
    t_rec = time.perf_counter()
    X, Y, rows, rec_stats = wsm.record(mesh, u, 0.0, w.dt, train_steps, every=every, capacity=cap, log=log, **opts)
    t_rec = time.perf_counter() - t_rec
    norms = wsm.standardise(X, Y, rows)
    net = Network(nin, nout, wsm.init_params(np.random.default_rng(0), nin, nout))
    t_tr = time.perf_counter()
    tr, va = wsm.train(net, X, Y, rows, epochs=epochs, batch=8192, lr=1e-3, log=log)
    torch.cuda.synchronize()
    t_tr = time.perf_counter() - t_tr
    del X, Y
    torch.cuda.empty_cache()
    mesh.warmstart_set(net, *norms)
    t0 = train_steps * w.dt
    eval_desc = "the %d steps after the training trajectory" % eval_steps
    if eval_seed is not None:
        we = workload("shell-p3" if w.p == 3 else "shell-p4", eval_seed)
        mesh.set_physics(we.phys)
        u = torch.from_numpy(shell_state(we, mesh.nodes().reshape(w.n_elem, -1, 3)).ravel()).to(u.device)
        t0 = 0.0
        eval_desc = "%d steps from t = 0 of the seed-%d workload (held out)" % (eval_steps, eval_seed)
    out = {"metric": "s per implicit step, learned/mixed vs plain @1e-8", "unit": "s", "higher_is_better": False,
           "config": {"workload": w.name, "n_dof": w.n_dof, "dt_s": 60.0, "train_steps": train_steps,
                      "train_rows": rows, "train_stages": 3 * train_steps, "eval_steps": eval_steps,
                      "eval": eval_desc, "epochs": epochs},
           "record_seconds": t_rec, "train_seconds": t_tr, "train_loss": tr, "val_loss": va}
    for prec in ("f64", "f32"):
        sp, sl, up, ul = wsm.compare(mesh, u, t0, w.dt, eval_steps, jvp_prec=prec, log=log, **opts)
        agg = lambda ss, k: float(np.mean([sum(s[k]) for s in ss]))
        out[prec] = {
            "plain": {"s_per_step": float(np.mean([s["seconds"] for s in sp])),
                      "newton": agg(sp, "newton_its"), "gmres": agg(sp, "gmres_its")},
            "learned": {"s_per_step": float(np.mean([s["seconds"] for s in sl])),
                        "newton": agg(sl, "newton_its"), "gmres": agg(sl, "gmres_its"),
                        "fallback_stages": int(sum(sum(s["fallback"]) for s in sl)),
                        "mean_guess_scale": float(np.mean([g for s in sl for g in s["guess_scale"]])),
                        "res0_over_plain": float(np.mean([a / b for s1, s2 in zip(sl, sp)
                                                          for a, b in zip(s1["res0"], s2["res0"]) if b > 0]))},
            "state_rel_diff": float(torch.linalg.norm(up - ul).item() / torch.linalg.norm(up - u).item()),
        }
        # what a guess must reach to save a Newton iteration: the plain guess starts at
        # rho = |G(U_p)| / |G(u_n)| and Newton takes k iterations to 1e-8, so one iteration is worth
        # a factor of about (1e-8 / rho)^(1/k) of the starting residual (geometric mean)
        rho_p = [a / b for s in sp for a, b in zip(s["res0"], s["ref"]) if b > 0]
        rho_l = [a / b for s in sl for a, b in zip(s["res0"], s["ref"]) if b > 0]
        k_p = out[prec]["plain"]["newton"] / 3.0
        gm_p = float(np.exp(np.mean(np.log(rho_p)))) if rho_p else None
        out[prec]["guess_residual"] = {
            "plain_res0_over_ref_geomean": gm_p,
            "learned_res0_over_ref_geomean": float(np.exp(np.mean(np.log(rho_l)))) if rho_l else None,
            "newton_per_stage_plain": k_p,
            "factor_one_iteration_is_worth": float((1e-8 / gm_p) ** (1.0 / k_p)) if gm_p else None,
            "note": "a guess saves a Newton iteration only if it lowers the starting stage residual by about "
                    "this factor relative to the plain guess; the learned guess lowers it by res0_over_plain"}
    out["value"] = out["f32"]["learned"]["s_per_step"]
    out["vs_plain_f64"] = out["f64"]["plain"]["s_per_step"] / out["value"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # R(u) takes ~0.17 ms: the defaults keep the GPU busy long enough (~60 ms of warm-up work)
    # to reach its sustained clock; 20 steps after 3 warm-ups read ~11% below steady state
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="shell-p3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-p4", action="store_true", help="skip the implicit steps on the 92M-DOF p = 4 shell")
    ap.add_argument("--preroll", type=float, default=0.3,
                    help="seconds of the same work before each timed loop (0 for counter runs)")
    ap.add_argument("--no-warmstart", action="store_true", help="skip the reduced warm-start experiment")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain device copy of known size (calibrates HBM counters)")
    ap.add_argument("--only", default="all", choices=["all", "residual", "implicit", "columns", "mfma"],
                    help="residual: only the R(u) timing; implicit: only the implicit steps; columns: only "
                         "the column batch; mfma: only the two matrix-core kernels, the BF16 J v and the "
                         "network's inference (for counter runs)")
    ap.add_argument("--implicit-runs", default="f64,f32,bf16,f32_rb4,f32_no_precond",
                    help="which implicit-step runs (with --only implicit)")
    ap.add_argument("--mode", default="default", choices=["default", "warmstart", "sweep"],
                    help="sweep: the parametric study of the 1D model (three cases x 75 columns)")
    ap.add_argument("--sweep-hours", type=float, default=72.0, help="model hours per case (sweep mode)")
    ap.add_argument("--sweep-quadrature", type=int, default=1, choices=(0, 1),
                    help="sweep mode: 1 over-integrated residual without a filter, 0 collocated with the filter")
    ap.add_argument("--sweep-serial", action="store_true",
                    help="sweep mode: run the cases one after another instead of concurrently")
    ap.add_argument("--implicit-steps", type=int, default=16)
    ap.add_argument("--all-pass1-configs", action="store_true",
                    help="with --only residual: time every element-pass launch configuration")
    ap.add_argument("--pass1-config", type=int, default=None, choices=range(6),
                    help="element-pass launch configuration instead of the autotuned one (for counter runs)")
    ap.add_argument("--ws-train-steps", type=int, default=60)
    ap.add_argument("--ws-eval-steps", type=int, default=8)
    ap.add_argument("--ws-epochs", type=int, default=8)
    ap.add_argument("--ws-every", type=int, default=4, help="record one element in this many per stage")
    ap.add_argument("--ws-eval-seed", type=int, default=None,
                    help="evaluate on a held-out trajectory of the workload drawn with this seed")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path", file=sys.stderr)
        raise SystemExit(2)

    import torch

    import synth
    from paper_2306_01085_amd import Mesh

    if args.mode == "sweep":
        from paper_2306_01085_amd import sweep
        out = {"metric": "parametric sweep of the 1D model: column-steps/s", "unit": "column-steps/s",
               "higher_is_better": True, "cases": []}
        ws = [synth.sweep_case(case) for case in (1, 2, 3)]
        kw = dict(hours=args.sweep_hours, quadrature=args.sweep_quadrature,
                  filter_rate=0.0 if args.sweep_quadrature else FILTER_RATE, log=log)
        if args.sweep_serial:
            results = [sweep.run_case(w, **kw) for w in ws]
            wall = sum(r["seconds"] for r in results)
        else:
            results, wall = sweep.run_cases(ws, **kw)
        for w, res in zip(ws, results):
            res["rho400_spread"] = sweep.summarise(w, res)
            del res["logrho_400km"]
            res.update({"f107bar": w.extra["fbar"], "day": w.extra["day"], "elements": int(w.nelem[0]), "p": 2})
            out["cases"].append(res)
        out["cases_run"] = "one after another" if args.sweep_serial else "concurrently, a stream per case"
        out["seconds"] = wall
        out["value"] = sum(c["columns"] * c["steps"] for c in out["cases"]) / wall
        print(json.dumps(out), flush=True)
        return

    if args.only == "columns":
        print(json.dumps(column_batch()[0]), flush=True)
        return

    dev = torch.device("cuda:0")
    w = workload(args.workload)
    log("building %s: %d elements, %d DOF" % (w.name, w.n_elem, w.n_dof))
    mesh = Mesh.shell(p=w.p, n_ang=w.n_ang, n_rad=w.n_rad, r_bot=w.r_bot, r_top=w.r_top, stretch=w.stretch,
                      phys=w.phys)
    X = mesh.nodes().reshape(w.n_elem, -1, 3)
    u_np = shell_state(w, X)
    u = torch.from_numpy(u_np.ravel()).to(dev)
    from paper_2306_01085_amd import autotune
    if args.pass1_config is not None:
        p1_cfg = args.pass1_config
        mesh.set_option("shell_pass1_config", p1_cfg)
    else:
        p1_cfg, _ = autotune.tune_shell_pass1(mesh, u)
    log("element-pass configuration %d" % p1_cfg)
    v = torch.from_numpy(synth.tangent(u_np.shape, 1).ravel()).to(dev)
    v32 = v.float()
    del u_np, X
    r = torch.empty_like(u)
    jv = torch.empty_like(u)
    jv32 = torch.empty_like(v32)
    t = 0.0

    def preroll(fn, preroll_s=None):
        # keep the GPU busy with the same work for preroll_s first: a timed region of a few
        # milliseconds right after lighter work catches the clock still rising (R read ~10%
        # slow over 20 evaluations after 3 warm-ups without it)
        t_end = time.perf_counter() + (args.preroll if preroll_s is None else preroll_s)
        while time.perf_counter() < t_end:
            for _ in range(10):
                fn()
            torch.cuda.synchronize()

    def timed(fn, steps, preroll_s=None):
        preroll(fn, preroll_s)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    if args.mode == "warmstart":
        del r, jv, jv32, v, v32
        print(json.dumps(warmstart_experiment(w, mesh, u, train_steps=args.ws_train_steps,
                                              eval_steps=args.ws_eval_steps, every=args.ws_every,
                                              epochs=args.ws_epochs, eval_seed=args.ws_eval_seed)), flush=True)
        return

    if args.only == "implicit":
        del r, jv, jv32, v, v32
        res = implicit_steps(w, mesh, u, args.implicit_steps, only=args.implicit_runs.split(","))
        if args.copy_probe:
            copy_probe(dev)
        print(json.dumps(res), flush=True)
        return

    f_r = lambda: mesh.residual(u, t, out=r)
    f_j64 = lambda: mesh.jvp(u, v, t, "f64", out=jv)
    f_j32 = lambda: mesh.jvp(u, v32, t, "f32", out=jv32)
    jvfd = torch.empty_like(jv)
    f_jfd = lambda: mesh.jvp(u, v, t, "f64_fd", out=jvfd)
    jvb = torch.empty_like(v32) if w.p in (3, 4) else None
    f_jb = (lambda: mesh.jvp(u, v32, t, "bf16", out=jvb)) if w.p in (3, 4) else None
    if args.only == "mfma":
        jvb = torch.empty_like(v32)
        ms_b = timed(lambda: mesh.jvp(u, v32, t, "bf16", out=jvb), args.steps)
        net = network_rates(w, args.steps, args.warmup, timed)
        print(json.dumps({"jvp_bf16_ms": ms_b, "jvp_bf16_gdofs": w.n_dof / ms_b / 1e6, "network": net}), flush=True)
        return
    if args.only == "residual":
        # with --all-pass1-configs every element-pass launch configuration runs in turn (one
        # counter run then covers them all: their kernels have distinct template names)
        cfgs = range(6) if args.all_pass1_configs else [p1_cfg]
        res = {}
        for cfg in cfgs:
            mesh.set_option("shell_pass1_config", cfg)
            for _ in range(args.warmup):
                f_r()
            ms_r = timed(f_r, args.steps)
            res[cfg] = {"residual_ms": ms_r, "gdofs": w.n_dof / ms_r / 1e6}
            log("configuration %d: %.4f ms" % (cfg, ms_r))
        if args.copy_probe:
            copy_probe(dev)
        print(json.dumps(res), flush=True)
        return
    for _ in range(args.warmup):
        f_r(); f_j64(); f_j32()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    ms_r = timed(f_r, args.steps)
    ms_j64 = timed(f_j64, args.steps)
    ms_j32 = timed(f_j32, args.steps)
    ms_jb = timed(f_jb, args.steps) if f_jb else None
    f_jfd()
    ms_jfd = timed(f_jfd, args.steps)
    # reduced-precision J v against the FP64 product (the FP64 product matches the oracle
    # to 1e-12 in the parity tests)
    nrm = torch.linalg.norm(jv).item()
    jv_err = {"f32": torch.linalg.norm(jv32.double() - jv).item() / nrm,
              "f64_fd": torch.linalg.norm(jvfd - jv).item() / nrm}
    if f_jb:
        f_jb()
        jv_err["bf16"] = torch.linalg.norm(jvb.double() - jv).item() / nrm
    ok = bool(torch.isfinite(r).all().item() and torch.isfinite(jv).all().item())
    # per-kernel event timing on the stream the kernels run on (the same pre-roll as the timed
    # regions: 20 evaluations right after the host-side norms above read the element pass
    # ~25% slow, the clock still rising; the trace pass, bound by HBM, hardly changes)
    preroll(f_r)
    mesh.profile(True)
    for _ in range(args.steps):
        f_r()
    prof = mesh.profile_read()
    mesh.profile(False)
    preroll(f_j64)
    mesh.profile(True)
    mesh.profile_read()
    for _ in range(args.steps):
        f_j64()
    prof.update(mesh.profile_read())
    mesh.profile(False)
    # the same products with the EUVAC heating (37 bins, Chapman optical depth) in place of
    # the prescribed profile: a state-dependent source evaluated at every node
    phys_e = dict(w.phys)
    phys_e.update(synth.euvac_physics(f107bar=150.0, day=80.0))
    phys_e["heating_model"] = 1
    phys_e["heat_amp"] = 0.0
    mesh.set_physics(phys_e)
    for _ in range(args.warmup):
        f_r(); f_j64(); f_j32()
    euv = {"residual_gdofs": w.n_dof / timed(f_r, args.steps) / 1e6,
           "jvp_f64_gdofs": w.n_dof / timed(f_j64, args.steps) / 1e6,
           "jvp_f32_gdofs": w.n_dof / timed(f_j32, args.steps) / 1e6,
           "heating": "EUVAC, F10.7bar 150, day 80, efficiency 0.25"}
    # and with the variable composition (fitted N2, O2, He fractions, O the balance): alone
    # with the prescribed heating, and together with EUVAC
    comp = {"fits": "synthetic two-exponential mass fractions (input generators)"}
    for key, base in (("prescribed_heating", w.phys), ("euvac", phys_e)):
        mesh.set_physics(dict(base, **synth.composition_physics()))
        for _ in range(args.warmup):
            f_r(); f_j64(); f_j32()
        comp[key] = {"residual_gdofs": w.n_dof / timed(f_r, args.steps) / 1e6,
                     "jvp_f64_gdofs": w.n_dof / timed(f_j64, args.steps) / 1e6,
                     "jvp_f32_gdofs": w.n_dof / timed(f_j32, args.steps) / 1e6}
    mesh.set_physics(w.phys)
    network = network_rates(w, args.steps, args.warmup, timed)
    if args.copy_probe:
        copy_probe(dev)
    ndof = w.n_dof
    p1_ms = prof["shell_pass1_R"][0] / prof["shell_pass1_R"][1]
    p2_ms = prof["shell_pass2_R"][0] / prof["shell_pass2_R"][1]
    b1 = pass1_bytes(w)
    fl1 = pass1_flops(w.p) * w.n_elem * (w.p + 1) ** 3
    tr_bytes, tr_detail = traffic(args.workload, p1_cfg)
    out = {
        "metric": "GDOF/s for DG R(u) & JVP; s per implicit step, learned/mixed vs plain @1e-8",
        "value": ndof / (ms_r * 1e-3) / 1e9,
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_r,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_dof": ndof, "n_elem": w.n_elem, "p": w.p, "fields": 5,
                   "step": "one R(u) evaluation", "pass1_config": p1_cfg},
        "jvp_f64_gdofs": ndof / (ms_j64 * 1e-3) / 1e9,
        "jvp_f32_gdofs": ndof / (ms_j32 * 1e-3) / 1e9,
        "jvp_bf16_gdofs": ndof / (ms_jb * 1e-3) / 1e9 if ms_jb else None,
        "jvp_f64_fd_gdofs": ndof / (ms_jfd * 1e-3) / 1e9,
        "jvp_rel_err_vs_f64": jv_err,
        "kernels_ms": {k: v_[0] / v_[1] for k, v_ in prof.items()},
        "residual_effective_gbs": residual_bytes(w) / (ms_r * 1e-3) / 1e9,
        "residual_target": {
            "reference_bytes_per_dof": R_REF_BYTES_PER_DOF,
            "hbm_frac_of_reference_roofline": R_REF_BYTES_PER_DOF * ndof / (ms_r * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "target_frac": HBM_TARGET_FRAC,
            "target_gdofs": HBM_TARGET_FRAC * HBM_PEAK_GBS / R_REF_BYTES_PER_DOF,
            "met": bool(R_REF_BYTES_PER_DOF * ndof / (ms_r * 1e-3) / 1e9 / HBM_PEAK_GBS >= HBM_TARGET_FRAC)},
        "roofline": element_pass_roofline(fl1, b1, p1_ms, tr_bytes, tr_detail,
                                          valu_counters(args.workload, p1_cfg, p1_ms)),
        "trace_pass": {"kernel": "shell_pass2 (R, f64)", "avg_launch_ms": p2_ms,
                       "algorithmic_bytes_per_launch": pass2_bytes(w),
                       "hbm_gbs_algorithmic": pass2_bytes(w) / (p2_ms * 1e-3) / 1e9,
                       "hbm_frac_algorithmic": pass2_bytes(w) / (p2_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "finite": ok,
    }
    log("implicit steps")
    out["euvac"] = euv
    out["composition"] = comp
    out["network"] = network
    out["implicit_step"] = implicit_steps(w, mesh, u, args.implicit_steps)
    del r, jv, jv32, v, v32, jvfd
    # the per-element network's BF16 tiles need 15 (p+1)^3 inputs a multiple of 8 and
    # 5 (p+1)^3 outputs a multiple of 32: p = 3 (960, 320); not p = 2 (405, 135) or p = 4 (1875, 625)
    ws_nin, ws_nout = 15 * (w.p + 1) ** 3, 5 * (w.p + 1) ** 3
    if not args.no_warmstart and (ws_nin % 8 or ws_nout % 32):
        out["warmstart"] = {"skipped": "per-element network of %d inputs and %d outputs at p = %d: the BF16 tiles "
                                       "need inputs a multiple of 8 and outputs a multiple of 32" % (ws_nin, ws_nout, w.p)}
    elif not args.no_warmstart:
        log("warm-start network: record, train, plain vs learned")
        ws = warmstart_experiment(w, mesh, u, train_steps=60, eval_steps=8, every=4, epochs=8)
        ws["scale"] = "reduced (60 recorded steps, 8 evaluation steps); bench.py --mode warmstart " \
                      "--ws-train-steps 667 --ws-eval-steps 200 --ws-eval-seed 1 is the configured scale"
        out["warmstart"] = ws
    del mesh, u
    torch.cuda.empty_cache()
    if not args.no_p4:
        log("implicit steps on the 92M-DOF p = 4 shell")
        out["implicit_step_p4"] = implicit_steps_shell("shell-p4", 5, ("f64", "f32"))
    log("column batch")
    out["columns"], col_samples = column_batch()
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        counts = {"shell-p3 (7.9M DOF), f64 J v, line preconditioner": (w.n_dof, out["implicit_step"]["f64"])}
        if "implicit_step_p4" in out and out["implicit_step_p4"]["f64"]["s_per_step"]:
            counts["shell-p4 (92M DOF), f64 J v, line preconditioner"] = (out["implicit_step_p4"]["n_dof"],
                                                                       out["implicit_step_p4"]["f64"])
        out["cpu_baseline"] = cpu_baseline(w, implicit=counts)
        # sampled columns of the batch: one oracle step each (timed with the baseline) and the
        # GPU batch's step against it
        cse = column_sample_error(col_samples)
        out["cpu_baseline"]["column_batch_sample"] = {
            "workload": "the smallest column of each degree in the 4096-column batch, one DIRK(3,3) step of "
                        "10 s, dense Newton 1e-9, 1 thread", "columns": cse}
        for name, rows in cse.items():
            out["columns"][name]["sampled_rel_err_vs_oracle"] = {str(r["column"]): r["rel_err_vs_oracle"]
                                                                 for r in rows}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
