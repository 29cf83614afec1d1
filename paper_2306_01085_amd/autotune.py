"""Autotuner of launch configurations, with a JSON cache.

tune_columns: picks the number of persistent wavefronts of dg_columns_integrate
for a column batch by timing short trial integrations (on a scratch copy of the
state) for each candidate; tune_columns_policy: then its chord-Jacobian rebuild
thresholds the same way; tune_shell_pass1: picks the element-pass configuration
of the shell residual by the time of whole residual evaluations. Results are
cached in a JSON file keyed by the workload's shape (DG_TUNE_CACHE, default
~/.cache/dgthermo_tuning.json) and re-applied without timing on later calls.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

_CACHE = os.environ.get("DG_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "dgthermo_tuning.json"))


def _load():
    try:
        with open(_CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(cache):
    try:
        os.makedirs(os.path.dirname(_CACHE), exist_ok=True)
        tmp = _CACHE + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, _CACHE)
    except OSError:
        pass


def columns_key(mesh):
    ne = np.asarray(mesh.col_nelem)
    pp = np.asarray(mesh.col_p)
    hist = [int(np.sum(ne[pp == p])) for p in (2, 3, 4)]
    return "columns:%d:%d:%d:%d" % (len(ne), *hist)


def tune_columns(mesh, u, t0, dt, steps=8, candidates=(256, 512, 1024, 2048, 4096), force=False, log=None, tag=""):
    """choose 'columns_grid' for this batch; returns (best grid, {grid: seconds}). tag: a
    label of the mesh's other settings (the quadrature) added to the cache key"""
    import torch
    key = columns_key(mesh) + tag
    cache = _load()
    if key in cache and not force:
        mesh.set_option("columns_grid", cache[key]["grid"])
        return cache[key]["grid"], cache[key].get("times", {})
    times = {}
    scratch = torch.empty_like(u)
    # an untimed call at the largest grid first: the workspace (per persistent wavefront) is
    # allocated there once, so no timed trial pays for growing it
    mesh.set_option("columns_grid", int(min(max(candidates), mesh.n_col)))
    scratch.copy_(u)
    mesh.columns_integrate(scratch, t0, dt, steps, raise_on_failure=False)
    torch.cuda.synchronize()
    for g in candidates:
        g = int(min(g, mesh.n_col)) if g > mesh.n_col else int(g)
        if str(g) in times:
            continue
        mesh.set_option("columns_grid", g)
        scratch.copy_(u)
        torch.cuda.synchronize()
        t = time.perf_counter()
        mesh.columns_integrate(scratch, t0, dt, steps, raise_on_failure=False)
        torch.cuda.synchronize()
        times[str(g)] = time.perf_counter() - t
        if log:
            log("columns_grid %d: %.3f s" % (g, times[str(g)]))
    best = int(min(times, key=times.get))
    mesh.set_option("columns_grid", best)
    cache[key] = {"grid": best, "times": times}
    _store(cache)
    return best, times


def tune_columns_policy(mesh, u, t0, dt, steps=32, candidates=((75, 5), (50, 3), (90, 6), (99, 12)), force=False,
                        log=None, tag=""):
    """choose the chord-Jacobian rebuild thresholds of the column batch ('columns_jac_slow_pct',
    'columns_jac_stale_its': rebuild within a stage when an iteration leaves |G| above that
    percentage of its previous value, and after a step with a stage of more iterations than
    that) by timing trials of `steps` steps at the mesh's current grid; they change iteration
    counts, not what each stage converges to. Returns ((slow_pct, stale_its), {label: seconds})"""
    import torch
    key = columns_key(mesh) + tag + ":policy"
    cache = _load()
    if key in cache and not force:
        best = tuple(cache[key]["policy"])
        mesh.set_option("columns_jac_slow_pct", best[0])
        mesh.set_option("columns_jac_stale_its", best[1])
        return best, cache[key].get("times", {})
    times = {}
    scratch = torch.empty_like(u)
    for slow, stale in candidates:
        mesh.set_option("columns_jac_slow_pct", slow)
        mesh.set_option("columns_jac_stale_its", stale)
        scratch.copy_(u)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = mesh.columns_integrate(scratch, t0, dt, steps, raise_on_failure=False)
        torch.cuda.synchronize()
        label = "%d/%d" % (slow, stale)
        # a policy that leaves more columns failed than the others is not a candidate
        times[label] = (time.perf_counter() - t, int((np.asarray(st) != 0).sum()))
        if log:
            log("columns chord policy %s: %.3f s, %d failed" % (label, *times[label]))
    fewest = min(f for _, f in times.values())
    label = min((k for k, v in times.items() if v[1] == fewest), key=lambda k: times[k][0])
    best = tuple(int(x) for x in label.split("/"))
    mesh.set_option("columns_jac_slow_pct", best[0])
    mesh.set_option("columns_jac_stale_its", best[1])
    cache[key] = {"policy": list(best), "times": times}
    _store(cache)
    return best, times


def tune_shell_pass1(mesh, u, t=0.0, reps=40, configs=range(6), force=False, log=None, warm_s=0.3):
    """choose 'shell_pass1_config' by the time of whole residual evaluations (element pass and
    trace pass: a configuration whose element pass is a little faster can leave the trace pass
    slower), timed with events around `reps` back-to-back evaluations per configuration

    The GPU is first kept busy with residual evaluations for warm_s seconds: timed while its
    clock still rises, the configurations tried first would read slower than they are."""
    key = "shell:%d:%d:%d" % (mesh.p, mesh.n_elem, mesh.n_dof)
    cache = _load()
    if key in cache and not force and cache[key].get("by") == "residual":
        mesh.set_option("shell_pass1_config", cache[key]["config"])
        return cache[key]["config"], cache[key].get("times", {})
    import torch
    r = torch.empty_like(u)
    t_end = time.perf_counter() + warm_s
    while time.perf_counter() < t_end:
        for _ in range(20):
            mesh.residual(u, t, out=r)
        torch.cuda.synchronize()
    times = {}
    for c in configs:
        mesh.set_option("shell_pass1_config", c)
        for _ in range(3):
            mesh.residual(u, t, out=r)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            mesh.residual(u, t, out=r)
        b.record()
        torch.cuda.synchronize()
        times[str(c)] = a.elapsed_time(b) / reps
        if log:
            log("shell_pass1_config %d: %.1f us per residual" % (c, 1e3 * times[str(c)]))
    best = int(min(times, key=times.get))
    mesh.set_option("shell_pass1_config", best)
    cache[key] = {"config": best, "times": times, "by": "residual"}
    _store(cache)
    return best, times
