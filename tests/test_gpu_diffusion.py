"""GPU parity of the p_s diffusion kappa* D_sa of eq. 1 (handles created with kappa_star > 0):
adaptation tendencies in both stage-kernel forms, steps, stage and step adjoints against the FP64
oracle with the same kappa*, and mass conservation."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2103_10114_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = ("U", "V", "Phi", "ps")
KSTAR = 2e5


def small(nx, ny, nz, seed=13, degree=5):
    return dataclasses.replace(synth.CONFIGS["c1"], nx=nx, ny=ny, nz=nz, degree=degree, seed=seed)


def _core(cfg, st, prec, **kw):
    from paper_2103_10114_amd import Dycore
    return Dycore(cfg.nx, cfg.ny, cfg.nz, cfg.dt, prec=prec, phis=st["phis"], kappa_star=KSTAR, **kw)


def _host(d):
    return {k: v.detach().cpu().numpy().astype(np.float64) for k, v in d.items() if k in KEYS}


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# 128 columns: the pipelined adaptation kernel; FP64 rows of 750 columns: the per-level form
@pytest.mark.parametrize("nxyz", [(128, 64, 9), (750, 8, 3)])
def test_diffusion_tendency_and_steps_fp64(nxyz):
    """The adaptation tendency and two outer steps with kappa* in FP64 equal the oracle's (1e-12,
    1e-11); the diffusion changes the p_s tendency."""
    cfg = small(*nxyz)
    st = synth.make_state(cfg)
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"], kstar=KSTAR)
    want = o.tendency(st, "A")
    plain = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"]).tendency(st, "A")
    core = _core(cfg, st, "fp64", forward_only=True)
    got = _host(core.tendency(core.to_device(st), "A"))
    for k in KEYS:
        assert _rel(got[k], want[k]) < 1e-12, (k, _rel(got[k], want[k]))
    print(f"diffusion share of the p_s tendency: {_rel(plain['ps'], want['ps']):.3e}", flush=True)
    assert _rel(plain["ps"], want["ps"]) > 1e-4
    ws = o.step(st, 2, cfg.dt)
    d = core.to_device(st)
    core.step(d, 2)
    gs = _host(d)
    for k in KEYS:
        assert _rel(gs[k], ws[k]) < 1e-11, (k, _rel(gs[k], ws[k]))


def test_diffusion_mass_conserved_c1():
    """C1 with kappa* in FP64: the flux form keeps the global mass to 1e-13 over 10 steps."""
    cfg = synth.CONFIGS["c1"]
    st = synth.make_state(cfg)
    core = _core(cfg, st, "fp64", forward_only=True)
    d = core.to_device(st)
    m0, _ = core.diagnostics(d)
    core.step(d, 10)
    m1, _ = core.diagnostics(d)
    assert abs(m1 - m0) / m0 < 1e-13


@pytest.mark.parametrize("nxyz", [(64, 32, 4), (130, 66, 5)])
def test_diffusion_adjoint_fp64(nxyz):
    """Stage adjoints (both processes) and the step adjoint with kappa* equal the oracle's."""
    cfg = small(*nxyz)
    st = synth.make_state(cfg)
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"], kstar=KSTAR)
    core = _core(cfg, st, "fp64")
    ao = synth.random_like(st, 51)
    ch = 200.0
    for process in "AL":
        wb, wi = o.adj_stage(st, ao, ch, process)
        d = core.to_device(st)
        a = core.to_device(ao)
        ab = {k: torch.zeros_like(v) for k, v in d.items()}
        ai = {k: torch.zeros_like(v) for k, v in d.items()}
        core.stage_adjoint(process, ch, d, a, ab, ai)
        gb, gi = _host(ab), _host(ai)
        for k in KEYS:
            assert _rel(gb[k], wb[k]) < 1e-12, (process, "base", k)
            assert _rel(gi[k], wi[k]) < 1e-12, (process, "in", k, _rel(gi[k], wi[k]))
    lam = synth.random_like(st, 52)
    want = o.adj_step(st, lam, cfg.dt)
    a = core.to_device(lam)
    core.step_adjoint(core.to_device(st), a)
    got = _host(a)
    for k in KEYS:
        assert _rel(got[k], want[k]) < 1e-11, (k, _rel(got[k], want[k]))


def test_diffusion_stage_fp32():
    """FP32 storage with FP64 sums: one adaptation stage with kappa* from the FP32-rounded state, the
    increment within 2e-3 of its scale (as without the diffusion)."""
    cfg = small(130, 66, 5)
    st = synth.make_state(cfg)
    st32 = {k: st[k].astype(np.float32).astype(np.float64) for k in KEYS}
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"], kstar=KSTAR)
    ch = 100.0
    want = o.stage(st32, st32, ch, "A")
    core = _core(cfg, st, "fp32", forward_only=True)
    d = core.to_device(st32)
    out = {k: torch.empty_like(v) for k, v in d.items()}
    got = _host(core.stage("A", ch, d, d, out))
    for k in KEYS:
        inc = want[k] - st32[k]
        scale = max(np.abs(inc).max(), np.abs(want[k]).max() * 1e-7)
        err = np.abs(got[k] - want[k]).max() / scale
        print(f"fp32 stage A with kappa* {k}: err/incr {err:.3e}", flush=True)
        assert err < 2e-3, (k, err)
