"""Write the full-size parity fixtures: the oracle's FP64 R(u) and J(u)v on a whole
benchmark shell, sampled on a fixed set of elements.

Usage (from the repository root):
  python tests/golden/make_fullsize.py shell-p3|shell-p4|shell-p3-mixture-euvac

The oracle evaluates eq. (DGformulation) on the complete mesh (the 6x16x16x16 p = 3 shell
with 7,864,320 DOF, or the 6x32x32x24 p = 4 shell with 92,160,000 DOF; the third fixture is
the p = 3 shell with the variable composition and EUVAC heating); the state is the
workload's seeded input at the oracle's own nodes, the tangent the seeded unit-norm
Gaussian, t = 0.25. Stored per sampled element: R, the per-node term scale
(|volume| + |lift| + |source|), J v and its linearised term scale (|d volume| + |d lift| +
|d source|, from the complex step of each part), all [5, N]. Only oracle/ and the input generators
are called. It takes minutes (about 3 for shell-p3) and several GB of memory.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import dg as odg  # noqa: E402
from oracle import jac as ojac  # noqa: E402
from oracle import mesh as omesh  # noqa: E402

T_EVAL = 0.25
TANGENT_SEED = 11


def workload(name):
    return synth.fullsize_workload(name)


def sample_elements(w, count):
    """first and last layer of panel corners and edges, plus seeded interior picks"""
    na, nr = w.n_ang, w.n_rad
    cell = lambda panel, i, j: (panel * na + j) * na + i
    picks = []
    for panel in range(6):
        for (i, j) in ((0, 0), (na - 1, na - 1), (na // 2, 0)):
            picks.append(cell(panel, i, j) * nr + (panel % 2) * (nr - 1))
    rng = np.random.default_rng(2306)
    while len(picks) < count:
        e = int(rng.integers(0, w.n_elem))
        if e not in picks:
            picks.append(e)
    return sorted(set(picks))[:count]


def main():
    name = sys.argv[1]
    count = 12 if name == "shell-p4" else 24
    w = workload(name)
    t0 = time.time()
    om = omesh.shell_mesh(w.p, w.n_ang, w.n_rad, w.r_bot, w.r_top, w.stretch)
    print("mesh %.0f s" % (time.time() - t0), flush=True)
    u = synth.shell_state_at(w, om.X)
    els = sample_elements(w, count)
    R, scale = odg.residual_parts(om, w.phys, u, T_EVAL)
    R, scale = R[els].copy(), scale[els].copy()
    print("R %.0f s" % (time.time() - t0), flush=True)
    v = synth.tangent(u.shape, TANGENT_SEED)
    J, jscale = ojac.jvp_parts(om, w.phys, u, v, T_EVAL)
    J, jscale = J[els].copy(), jscale[els].copy()
    print("J v %.0f s" % (time.time() - t0), flush=True)
    out = {
        "what": "oracle FP64 R(u) and J(u)v on the full %s workload (eq. DGformulation), sampled elements" % name,
        "workload": name, "p": w.p, "n_ang": w.n_ang, "n_rad": w.n_rad, "n_dof": int(u.size),
        "t": T_EVAL, "tangent_seed": TANGENT_SEED, "elements": els,
        "R": R.tolist(), "scale": scale.tolist(), "Jv": J.tolist(), "jv_scale": jscale.tolist(),
    }
    path = os.path.join(ROOT, "tests", "golden", "fullsize_%s.json" % name)
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
