"""Full-size parity of R(u) and J(u)v on the benchmark shells (6x16x16x16 p = 3, 7.9M DOF;
6x32x32x24 p = 4, 92M DOF; the p = 3 shell with the variable composition and EUVAC heating,
which runs the extended-physics instantiation) against the oracle's FP64 values on
sampled elements.

The expected values are tests/golden/fullsize_<workload>.json, written by
tests/golden/make_fullsize.py from oracle/ and the input generators only (the oracle
evaluates the whole mesh; a fixture keeps whole sampled elements, corners and edges of
the cube panels, bottom and top layers among them). The GPU evaluates the same seeded
state at its own nodes (the two node sets agree to round-off), in every launch
configuration of the element pass, so the one the bench's autotuner picks is covered.
Bounds: R within 1e-12 of the sampled term scale (|volume| + |lift| + |source|); J v FP64
within 1e-12 of the sampled linearised term scale (|d volume| + |d lift| + |d source|) and
within 1e-11 relative in the 2-norm over the samples (the tangent is unit-norm over 7.9M or
92M entries, so the sampled products are small); FP32 within 1e-5; the BF16-MFMA product within 3e-2."""
import json
import os

import numpy as np
import pytest

import synth
from gpu_common import need_gpu, to_dev, torch

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name", ["shell-p3", "shell-p4", "shell-p3-mixture-euvac"])
def test_fullsize_residual_and_jvp(name):
    need_gpu()
    from paper_2306_01085_amd import Mesh
    path = os.path.join(GOLDEN, "fullsize_%s.json" % name)
    if not os.path.exists(path):
        pytest.skip("fixture %s not written (python tests/golden/make_fullsize.py %s)" % (path, name))
    with open(path) as f:
        fx = json.load(f)
    w = synth.fullsize_workload(name)
    assert (w.p, w.n_ang, w.n_rad) == (fx["p"], fx["n_ang"], fx["n_rad"])
    gm = Mesh.shell(p=w.p, n_ang=w.n_ang, n_rad=w.n_rad, r_bot=w.r_bot, r_top=w.r_top, stretch=w.stretch,
                    phys=w.phys)
    N = (w.p + 1) ** 3
    u = synth.shell_state_at(w, gm.nodes().reshape(w.n_elem, N, 3))
    assert u.size == fx["n_dof"]
    v = synth.tangent(u.shape, fx["tangent_seed"])
    ut, vt = to_dev(u), to_dev(v)
    del v
    els = np.asarray(fx["elements"])
    R_ref, scale, J_ref = (np.asarray(fx[k]) for k in ("R", "scale", "Jv"))
    t = fx["t"]

    def sampled(x):
        return x.reshape(w.n_elem, 5, N)[torch.as_tensor(els, device=x.device)].double().cpu().numpy()

    # (a mesh with EUVAC or the composition runs its one extended instantiation whatever the
    # configuration: one pass suffices)
    for cfg in (range(6) if w.phys.get("heating_model", 0) == 0 and not w.phys.get("composition") else [0]):
        gm.set_option("shell_pass1_config", cfg)
        r = sampled(gm.residual(ut, t=t))
        err = np.max(np.abs(r - R_ref)) / np.max(scale)
        assert err < 1e-12, (name, cfg, err)
        j32 = sampled(gm.jvp(ut, vt.float(), t=t, prec="f32"))
        e32 = np.linalg.norm(j32 - J_ref) / np.linalg.norm(J_ref)
        assert e32 < 1e-5, (name, cfg, e32)
    j64 = sampled(gm.jvp(ut, vt, t=t))
    e64 = np.linalg.norm(j64 - J_ref) / np.linalg.norm(J_ref)
    assert e64 < 1e-11, (name, e64)
    if "jv_scale" in fx:
        el64 = np.max(np.abs(j64 - J_ref)) / np.max(np.asarray(fx["jv_scale"]))
        assert el64 < 1e-12, (name, el64)
    if w.p in (3, 4):
        jb = sampled(gm.jvp(ut, vt.float(), t=t, prec="bf16"))
        eb = np.linalg.norm(jb - J_ref) / np.linalg.norm(J_ref)
        assert eb < 3e-2, (name, eb)
    print(name, "R", err, "J v FP64", e64, "FP32", e32, "BF16", eb)
