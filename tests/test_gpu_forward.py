"""GPU parity of the forward stage and step kernels against the FP64 oracle (through the C-ABI)."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2103_10114_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _core(cfg, st, prec, **kw):
    from paper_2103_10114_amd import Dycore
    return Dycore(cfg.nx, cfg.ny, cfg.nz, cfg.dt, prec=prec, phis=st["phis"], **kw)


def _host(d):
    return {k: v.detach().cpu().numpy().astype(np.float64) for k, v in d.items()}


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def small(nx, ny, nz, seed=3, degree=5):
    return dataclasses.replace(synth.CONFIGS["c1"], nx=nx, ny=ny, nz=nz, degree=degree, seed=seed)


GRIDS = [small(16, 8, 3), small(40, 20, 4), small(130, 66, 5), synth.CONFIGS["c1"]]


@pytest.mark.parametrize("cfg", GRIDS, ids=lambda c: f"{c.nx}x{c.ny}x{c.nz}")
@pytest.mark.parametrize("process", ["A", "L"])
def test_tendency_fp64(cfg, process):
    """Single-stage tendency T(in) in FP64 mode equals the oracle to 1e-12 (relative to max |T|)."""
    print(f"tendency fp64 {cfg.nx}x{cfg.ny}x{cfg.nz} {process}", flush=True)
    st = synth.make_state(cfg)
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"])
    want = o.tendency(st, process)
    core = _core(cfg, st, "fp64", forward_only=True)
    got = _host(core.tendency(core.to_device(st), process))
    for k in ("U", "V", "Phi", "ps"):
        if np.abs(want[k]).max() == 0:
            assert np.abs(got[k]).max() == 0
            continue
        assert _rel(got[k], want[k]) < 1e-12, (k, _rel(got[k], want[k]))


@pytest.mark.parametrize("block", [64, 128, 256])
def test_tendency_fp64_blocks(block):
    """Results do not depend on the advection tiles' workgroup size (64 and 128 threads turn the
    rows next to the poles into wide tiles)."""
    cfg = small(150, 32, 4)
    st = synth.make_state(cfg)
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"])
    core = _core(cfg, st, "fp64", forward_only=True, block=block)
    for process in "AL":
        want = o.tendency(st, process)
        got = _host(core.tendency(core.to_device(st), process))
        for k in ("U", "V", "Phi"):
            assert _rel(got[k], want[k]) < 1e-12, (process, k)


@pytest.mark.parametrize("cfg", GRIDS[:3], ids=lambda c: f"{c.nx}x{c.ny}x{c.nz}")
def test_step_fp64(cfg):
    """Whole outer steps (3M adaptation + 3 advection stages) in FP64 match the oracle."""
    print(f"step fp64 {cfg.nx}x{cfg.ny}x{cfg.nz}", flush=True)
    st = synth.make_state(cfg)
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"])
    want = o.step(st, 3, cfg.dt)
    core = _core(cfg, st, "fp64", forward_only=True)
    assert core.substeps == o.substeps(cfg.dt)
    d = core.to_device(st)
    core.step(d, 3)
    got = _host(d)
    for k in ("U", "V", "Phi", "ps"):
        assert _rel(got[k], want[k]) < 1e-11, (k, _rel(got[k], want[k]))
    assert np.all(got["U"][0] == 0) and np.all(got["U"][-1] == 0)


def test_c1_20_steps_fp64():
    """C1 (128x64x9, dt 600 s, 20 steps) in FP64: per-field error <= 1e-12 relative; mass conserved."""
    cfg = synth.CONFIGS["c1"]
    st = synth.make_state(cfg)
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"])
    want = o.step(st, cfg.steps, cfg.dt)
    core = _core(cfg, st, "fp64", forward_only=True)
    d = core.to_device(st)
    m0, _ = core.diagnostics(d)
    core.step(d, cfg.steps)
    m1, _ = core.diagnostics(d)
    got = _host(d)
    for k in ("U", "V", "Phi", "ps"):
        l2 = np.linalg.norm(got[k] - want[k]) / np.linalg.norm(want[k])
        print(f"c1 fp64 {k}: rel-L2 {l2:.3e} max {_rel(got[k], want[k]):.3e}")
        assert l2 < 1e-12 and _rel(got[k], want[k]) < 1e-12
    assert abs(m1 - m0) / m0 < 1e-13


@pytest.mark.parametrize("process", ["A", "L"])
def test_stage_fp32(process):
    """FP32 bulk / FP64 accumulation: one stage from an FP32-rounded state against the FP64 oracle."""
    cfg = small(130, 66, 5)
    st = synth.make_state(cfg)
    st32 = {k: st[k].astype(np.float32).astype(np.float64) for k in ("U", "V", "Phi", "ps")}
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"])
    ch = 100.0
    want = o.stage(st32, st32, ch, process)
    core = _core(cfg, st, "fp32", forward_only=True)
    d = core.to_device(st32)
    out = {k: torch.empty_like(v) for k, v in d.items()}
    got = _host(core.stage(process, ch, d, d, out))
    for k in ("U", "V", "Phi", "ps"):
        # the increment ch*T carries the FP32 error; compare it to the increment scale
        inc = want[k] - st32[k]
        scale = max(np.abs(inc).max(), np.abs(want[k]).max() * 1e-7)
        err = np.abs(got[k] - want[k]).max() / scale
        print(f"fp32 stage {process} {k}: err/incr {err:.3e}")
        assert err < 2e-3, (k, err)
