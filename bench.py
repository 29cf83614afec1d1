"""Benchmark of the DG thermosphere hot path on one MI355X.

Default workload: the cubed-sphere shell 6 x 16 x 16 angular x 16 radial elements
(stretch 1.15), p = 3, 5 fields: 24,576 elements, 7,864,320 DOF. A step is one
evaluation of the residual R(u) (the operator every Newton, GMRES and DIRK stage
is built from); J(u)v in FP64 and FP32 is timed the same way and reported beside
it. Inputs are resident in HBM before the timed region. Prints one JSON line.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload shell-p3|shell-p4]
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name):
    import synth
    if name == "shell-p3":
        return synth.config_shell_p3(0)
    if name == "shell-p4":
        return synth.config_shell_p4(0)
    raise SystemExit("unknown workload %s" % name)


def shell_state(w, X):
    """state at the library's nodes X [E, N, 3] (element e = cell * n_rad + layer, node
    j = cz * n^2 + angular node): angular directions are shared by every layer and
    every radial node of a cell, so the separable generator runs on (cell, angular
    node) x (layer, cz)"""
    import synth
    n = w.p + 1
    N2 = n * n
    A = 6 * w.n_ang ** 2
    Xg = X.reshape(A, w.n_rad, n, N2, 3)
    unit = Xg[:, 0, 0] / np.linalg.norm(Xg[:, 0, 0], axis=-1, keepdims=True)      # [A, N2, 3]
    radii = np.linalg.norm(Xg[0, :, :, 0], axis=-1)                               # [n_rad, n]
    u = synth.shell_state_product(w.T_inf, w.pert, unit.reshape(-1, 3), radii.ravel())   # [5, A*N2, n_rad*n]
    u = u.reshape(5, A, N2, w.n_rad, n)
    return np.ascontiguousarray(np.transpose(u, (1, 3, 0, 4, 2))).reshape(A * w.n_rad, 5, n * N2)


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


def residual_bytes(w):
    """algorithmic HBM bytes of one full R(u) (both passes): pass 1 as above; pass 2
    reads the neighbours' traces and face-node states and updates R on face nodes"""
    n = w.p + 1
    N, N2 = n ** 3, n ** 2
    Nface = N - (n - 2) ** 3
    E = w.n_elem
    p2 = E * (6 * 5 * N2 * 8 + 5 * N * 8 + 2 * 5 * Nface * 8)
    return pass1_bytes(w) + p2


def cpu_baseline(w, budget_s=20.0):
    """the FP64 oracle's residual on a bounded sample of the same workload: the same
    element type, degree and physics on a shell of 6 x 4 x 4 x 16 elements"""
    from threadpoolctl import threadpool_limits

    from oracle import dg as odg
    from oracle import mesh as omesh
    n_ang, n_rad = 4, w.n_rad
    om = omesh.shell_mesh(w.p, n_ang, n_rad, w.r_bot, w.r_top, w.stretch)
    u = np.moveaxis(w.state_fn()(om.X), 0, 1).copy()
    ndof = u.size
    times = []
    with threadpool_limits(limits=1):
        odg.residual(om, w.phys, u, 0.0)            # warm-up
        t_end = time.perf_counter() + budget_s
        while len(times) < 5 and time.perf_counter() < t_end:
            t0 = time.perf_counter()
            odg.residual(om, w.phys, u, 0.0)
            times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    return {"value": ndof / med / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
            "sample": "R(u) of the oracle on a 6x%dx%dx%d p=%d shell (%d DOF), median of %d runs, 1 BLAS thread"
                      % (n_ang, n_ang, n_rad, w.p, ndof, len(times))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="shell-p3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain device copy of known size (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        raise SystemExit(2)

    import torch

    import synth
    from paper_2306_01085_amd import Mesh

    dev = torch.device("cuda:0")
    w = workload(args.workload)
    log("building %s: %d elements, %d DOF" % (w.name, w.n_elem, w.n_dof))
    mesh = Mesh.shell(p=w.p, n_ang=w.n_ang, n_rad=w.n_rad, r_bot=w.r_bot, r_top=w.r_top, stretch=w.stretch,
                      phys=w.phys)
    X = mesh.nodes().reshape(w.n_elem, -1, 3)
    u_np = shell_state(w, X)
    u = torch.from_numpy(u_np.ravel()).to(dev)
    v = torch.from_numpy(synth.tangent(u_np.shape, 1).ravel()).to(dev)
    v32 = v.float()
    del u_np, X
    r = torch.empty_like(u)
    jv = torch.empty_like(u)
    jv32 = torch.empty_like(v32)
    t = 0.0

    def timed(fn, steps):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    f_r = lambda: mesh.residual(u, t, out=r)
    f_j64 = lambda: mesh.jvp(u, v, t, "f64", out=jv)
    f_j32 = lambda: mesh.jvp(u, v32, t, "f32", out=jv32)
    for _ in range(args.warmup):
        f_r(); f_j64(); f_j32()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    ms_r = timed(f_r, args.steps)
    ms_j64 = timed(f_j64, args.steps)
    ms_j32 = timed(f_j32, args.steps)
    ok = bool(torch.isfinite(r).all().item() and torch.isfinite(jv).all().item())
    # per-kernel event timing on the stream the kernels run on
    mesh.profile(True)
    for _ in range(args.steps):
        f_r()
    prof = mesh.profile_read()
    for _ in range(args.steps):
        f_j64()
    prof.update(mesh.profile_read())
    mesh.profile(False)
    if args.copy_probe:
        src = torch.empty(2 ** 28 // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    ndof = w.n_dof
    p1_ms = prof["shell_pass1_R"][0] / prof["shell_pass1_R"][1]
    p2_ms = prof["shell_pass2_R"][0] / prof["shell_pass2_R"][1]
    b1 = pass1_bytes(w)
    achieved = b1 / (p1_ms * 1e-3) / 1e9
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
                   "step": "one R(u) evaluation"},
        "jvp_f64_gdofs": ndof / (ms_j64 * 1e-3) / 1e9,
        "jvp_f32_gdofs": ndof / (ms_j32 * 1e-3) / 1e9,
        "kernels_ms": {k: v_[0] / v_[1] for k, v_ in prof.items()},
        "residual_effective_gbs": residual_bytes(w) / (ms_r * 1e-3) / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "shell_pass1 (R, f64)",
                     "algorithmic_bytes_per_launch": b1, "avg_launch_ms": p1_ms},
        "finite": ok,
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
