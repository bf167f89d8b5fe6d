"""GPU parity of the low-latitude filters (Sec. III-B, Table IV rows 1-2) that close each outer step
when a handle is created with DYCORE_LOWLAT_FILTERS: steps, the step adjoint, the recorded step and
batched members against the FP64 oracle with the same filters."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2103_10114_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = ("U", "V", "Phi", "ps")


def _core(cfg, st, prec, **kw):
    from paper_2103_10114_amd import Dycore
    return Dycore(cfg.nx, cfg.ny, cfg.nz, cfg.dt, prec=prec, phis=st["phis"], filters=True, **kw)


def _host(d):
    return {k: v.detach().cpu().numpy().astype(np.float64) for k, v in d.items() if k in KEYS}


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_filtered_steps_fp64_c1():
    """C1 (128x64x9), 5 filtered steps in FP64: within 1e-11 of the oracle's filtered steps, which
    differ from unfiltered ones (the filters act)."""
    cfg = synth.CONFIGS["c1"]
    st = synth.make_state(cfg)
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"], filters=True)
    want = o.step(st, 5, cfg.dt)
    plain = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"]).step(st, 5, cfg.dt)
    core = _core(cfg, st, "fp64", forward_only=True)
    d = core.to_device(st)
    core.step(d, 5)
    got = _host(d)
    for k in KEYS:
        err = _rel(got[k], want[k])
        print(f"filtered C1 fp64 {k}: {err:.3e} (filter effect {_rel(plain[k], want[k]):.3e})", flush=True)
        assert err < 1e-11, (k, err)
    assert _rel(plain["V"], want["V"]) > 1e-8


def test_filtered_steps_fp32_c2():
    """C2 (256x128x30), 10 filtered steps in FP32 from the FP32-rounded state against the oracle's
    filtered steps: per-field rel-L2 and max error, bounded like the unfiltered FP32 runs."""
    cfg = synth.CONFIGS["c2"]
    st = synth.make_state(cfg)
    st32 = {k: st[k].astype(np.float32).astype(np.float64) for k in KEYS}
    want = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"], filters=True).step(st32, 10, cfg.dt)
    core = _core(cfg, st, "fp32", forward_only=True)
    d = core.to_device(st32)
    core.step(d, 10)
    got = _host(d)
    for k in KEYS:
        l2 = np.linalg.norm(got[k] - want[k]) / np.linalg.norm(want[k])
        mx = _rel(got[k], want[k])
        print(f"filtered C2 fp32 10 steps {k}: rel-L2 {l2:.3e} max {mx:.3e}", flush=True)
        assert l2 < 9e-5 and mx < 1.75e-4, k


@pytest.mark.parametrize("nxyz", [(64, 32, 4), (130, 66, 5)])
def test_filtered_step_adjoint_fp64(nxyz):
    """The adjoint of a filtered step (the filters applied to the output adjoint first) equals the
    oracle's within 1e-11; the recorded forward equals dycore_step bit for bit and the recorded
    adjoint equals the recomputing one bit for bit."""
    nx, ny, nz = nxyz
    cfg = dataclasses.replace(synth.CONFIGS["c1"], nx=nx, ny=ny, nz=nz, degree=5, seed=17)
    st = synth.make_state(cfg)
    o = oracle.Oracle(nx, ny, nz, phis=st["phis"], filters=True)
    lam0 = synth.random_like(st, 91)
    want = o.adj_step(st, lam0, cfg.dt)
    core = _core(cfg, st, "fp64")
    a = core.to_device(lam0)
    core.step_adjoint(core.to_device(st), a)
    got = _host(a)
    for k in KEYS:
        assert _rel(got[k], want[k]) < 1e-11, (k, _rel(got[k], want[k]))
    x = core.to_device(st)
    y = core.to_device(st)
    core.step(x, 1)
    core.step_record(y)
    l2 = core.to_device(lam0)
    core.step_adjoint_recorded(l2)
    torch.cuda.synchronize()
    for k in KEYS:
        assert torch.equal(x[k], y[k]), k
        assert torch.equal(l2[k], a[k]), k


def test_filtered_batch_bitwise():
    """A batch of filtered and unfiltered members equals per-member steps bit for bit."""
    from paper_2103_10114_amd import Batch, Dycore
    cfgs = [dataclasses.replace(synth.CONFIGS["c1"], nx=64, ny=32, nz=5, degree=5, seed=31),
            dataclasses.replace(synth.CONFIGS["c1"], seed=32)]
    cores, states, refs = [], [], []
    for q, cfg in enumerate(cfgs):
        st = synth.make_state(cfg)
        c = Dycore(cfg.nx, cfg.ny, cfg.nz, cfg.dt, prec="fp32", phis=st["phis"], forward_only=True,
                   filters=(q == 0))
        cores.append(c)
        states.append(c.to_device(st))
        refs.append(c.to_device(st))
    b = Batch(cores, states)
    b.step(2)
    for c, r in zip(cores, refs):
        c.step(r, 2)
    torch.cuda.synchronize()
    for s, r in zip(states, refs):
        for k in KEYS:
            assert torch.equal(s[k], r[k]), k
