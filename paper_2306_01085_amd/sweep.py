"""The parametric study of the 1D model (section 4.3) as a batch workflow over the
library: for each solar-activity case, every (EUV efficiency, conductivity multiplier)
pair at each site is one column of a single column mesh, and all of them advance
together in persistent launches of dg_columns_integrate (DIRK(2,2), 30 s steps, EUVAC
heating with the zenith angle of each site, per-column efficiency and conductivity);
run_cases advances several cases concurrently, a stream per case.
Timing is the point; the density near 400 km at the end summarises what the grid spans.
"""
from __future__ import annotations

import time

import numpy as np


def initial_state(w, gm):
    """the workload's column states at the mesh's nodes, concatenated"""
    r = gm.nodes()
    off = gm.col_offsets()
    parts = []
    for c in range(gm.n_col):
        rc = r[off[c] // 3:off[c + 1] // 3].reshape(int(w.nelem[c]), int(w.p[c]) + 1)
        parts.append(np.moveaxis(w.state(c, rc), 0, 1).ravel())
    return np.concatenate(parts), r, off


def prepare_case(w, quadrature=1):
    """the case's column mesh (quadrature 1: the over-integrated residual, the weak form of
    eq. (DGformulation) with p + 2 Gauss points, no filter needed; 0: GLL collocation, which
    needs the modal filter against its growing intra-element mode) and its initial state on
    the device"""
    import torch

    from . import Mesh
    gm = Mesh.columns(w.nelem, w.p, w.r_bot, w.r_top, w.stretch, w.phys, w.col_phys)
    gm.set_option("column_quadrature", quadrature)
    u0, r, off = initial_state(w, gm)
    return gm, torch.from_numpy(u0).cuda(), r, off


def advance_case(w, gm, u, hours=72.0, chunk_hours=6.0, filter_rate=0.0, log=None, stream=None):
    """advance every column of the case `hours` of model time in chunks of persistent
    launches on `stream` (None: the current stream); returns (seconds, steps, Newton
    iterations, failed columns)"""
    import torch
    sync = torch.cuda.synchronize if stream is None else stream.synchronize
    step_s = 30.0
    n_total = int(round(hours * 3600.0 / step_s))
    chunk = max(1, int(round(chunk_hours * 3600.0 / step_s)))
    t = 0.0
    done = 0
    seconds = 0.0
    newton = 0
    failed = np.zeros(gm.n_col, dtype=bool)
    while done < n_total:
        k = min(chunk, n_total - done)
        sync()
        t0 = time.perf_counter()
        its, st = gm.columns_integrate(u, t, w.dt, k, scheme=22, newton_rtol=1e-8, max_newton=20,
                                       filter_rate=filter_rate, stream=stream, raise_on_failure=False)
        sync()
        seconds += time.perf_counter() - t0
        failed |= np.asarray(st) != 0
        newton += int(np.sum(its))
        done += k
        t += k * w.dt
        if log:
            log("%s: %.1f of %.1f h, %d columns failed" % (w.name, done * step_s / 3600.0, hours, int(failed.sum())))
    return seconds, n_total, newton, failed


def case_result(w, gm, u, r, off, hours, quadrature, filter_rate, seconds, n_total, newton, failed):
    """timing, failures and the log-density at the node nearest 400 km of each column"""
    uf = u.cpu().numpy()
    z400 = []
    for c in range(gm.n_col):
        rc = r[off[c] // 3:off[c + 1] // 3]
        j = int(np.argmin(np.abs(rc - w.extra["r400"])))
        e, a = divmod(j, int(w.p[c]) + 1)
        z400.append(float(uf[off[c] + e * 3 * (int(w.p[c]) + 1) + a]))
    return {"case": w.name, "columns": gm.n_col, "dof": gm.n_dof, "steps": n_total, "model_hours": hours,
            "quadrature": "p + 2 Gauss points" if quadrature else "GLL collocation", "filter_rate": filter_rate,
            "seconds": seconds, "column_steps_per_s": gm.n_col * n_total / seconds,
            "newton_per_column_step": newton / (gm.n_col * n_total), "failed": int(failed.sum()),
            "logrho_400km": z400}


def run_case(w, hours=72.0, chunk_hours=6.0, quadrature=1, filter_rate=0.0, log=None):
    """one case on its own: advance every column `hours` of model time; returns timing,
    failures and the log-density at the node nearest 400 km of each column at the end"""
    gm, u, r, off = prepare_case(w, quadrature)
    adv = advance_case(w, gm, u, hours, chunk_hours, filter_rate, log)
    return case_result(w, gm, u, r, off, hours, quadrature, filter_rate, *adv)


def run_cases(ws, hours=72.0, chunk_hours=6.0, quadrature=1, filter_rate=0.0, log=None):
    """every case at once. A case is a few dozen columns, one wavefront each, far fewer than
    the chip's 256 compute units; each case's mesh advances on a stream of its own, driven
    by a host thread of its own (the library call releases the interpreter while it waits
    for its stream), so the cases' launches share the chip instead of running one after
    another. Returns (the per-case results, as run_case's, each with its own seconds, and
    the wall time of them all)."""
    import threading

    import torch
    prep = [prepare_case(w, quadrature) for w in ws]
    streams = [torch.cuda.Stream() for _ in ws]
    adv = [None] * len(ws)
    errors = []

    def work(i):
        try:
            with torch.cuda.stream(streams[i]):
                adv[i] = advance_case(ws[i], prep[i][0], prep[i][1], hours, chunk_hours, filter_rate, log,
                                      stream=streams[i])
        except BaseException as e:   # re-raised below, in the calling thread
            errors.append(e)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(ws))]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if errors:
        raise errors[0]
    res = [case_result(w, gm, u, r, off, hours, quadrature, filter_rate, *a)
           for w, (gm, u, r, off), a in zip(ws, prep, adv)]
    return res, wall


def summarise(w, res):
    """per site: the spread of the density near 400 km over the (efficiency,
    conductivity) grid, relative to the nominal pair (0.25, 0.75)"""
    combos = w.extra["combos"]
    out = {}
    lr = np.asarray(res["logrho_400km"])
    for site in dict.fromkeys(s for s, _, _ in combos):
        idx = [i for i, (s, _, _) in enumerate(combos) if s == site]
        nom = [i for i in idx if combos[i][1] == 0.25 and combos[i][2] == 0.75][0]
        rel = np.exp(lr[idx] - lr[nom])
        out[site] = {"rho400_min_over_nominal": float(rel.min()), "rho400_max_over_nominal": float(rel.max())}
    return out
