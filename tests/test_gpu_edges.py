"""GPU edge cases: row lengths around the former whole-row LDS limits and the longest rows accepted
(every stage now runs in zonal tiles), the tilings of the row-fused stage adjoints, ragged tiles, a
single sigma level, zero steps, sizes the library refuses, and a stage adjoint whose base and input
adjoints are one buffer."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2103_10114_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def small(nx, ny, nz, seed=7, degree=4):
    return dataclasses.replace(synth.CONFIGS["c1"], nx=nx, ny=ny, nz=nz, degree=degree, seed=seed)


def _core(cfg, st, prec, **kw):
    from paper_2103_10114_amd import Dycore
    return Dycore(cfg.nx, cfg.ny, cfg.nz, cfg.dt, prec=prec, phis=st["phis"], **kw)


def _host(d):
    return {k: v.detach().cpu().numpy().astype(np.float64) for k, v in d.items()}


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# Row lengths at which whole-row kernels with 27 LDS rows would stop fitting 160 KiB (749/750 columns
# in FP64, 1498/1499 in FP32): the zonal tiles do not depend on them, and these cases check so.
@pytest.mark.parametrize("nx", [749, 750])
@pytest.mark.parametrize("process", ["A", "L"])
def test_tendency_fp64_across_pipeline_limit(nx, process):
    """Stage tendencies on rows of 749 and 750 columns (ragged last tiles) equal the oracle."""
    print(f"tendency fp64 nx={nx} {process}", flush=True)
    cfg = small(nx, 8, 3)
    st = synth.make_state(cfg)
    want = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"]).tendency(st, process)
    core = _core(cfg, st, "fp64", forward_only=True)
    got = _host(core.tendency(core.to_device(st), process))
    for k in ("U", "V", "Phi", "ps"):
        if np.abs(want[k]).max() == 0:
            assert np.abs(got[k]).max() == 0
            continue
        assert _rel(got[k], want[k]) < 1e-12, (k, _rel(got[k], want[k]))


@pytest.mark.parametrize("nx", [1000, 1498, 1499])
@pytest.mark.parametrize("process", ["A", "L"])
def test_stage_fp32_ragged_and_limit(nx, process):
    """FP32 stages on rows of 1000, 1498 and 1499 columns (ragged last tiles) within 2e-3 of the
    increment scale of the oracle's."""
    print(f"stage fp32 nx={nx} {process}", flush=True)
    cfg = small(nx, 10, 3)
    st = synth.make_state(cfg)
    st32 = {k: st[k].astype(np.float32).astype(np.float64) for k in ("U", "V", "Phi", "ps")}
    ch = 100.0
    want = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"]).stage(st32, st32, ch, process)
    core = _core(cfg, st, "fp32", forward_only=True)
    d = core.to_device(st32)
    out = {k: torch.empty_like(v) for k, v in d.items()}
    got = _host(core.stage(process, ch, d, d, out))
    for k in ("U", "V", "Phi", "ps"):
        inc = want[k] - st32[k]
        scale = max(np.abs(inc).max(), np.abs(want[k]).max() * 1e-7)
        err = np.abs(got[k] - want[k]).max() / scale
        assert err < 2e-3, (k, err)


# The tiled row-fused adaptation adjoint cuts rows into zonal tiles of <= 320 slots, halos included:
# Adaptation (halo n + 1): 731 columns give three tiles with a ragged last one; 96 columns one tile
# per row; at 512 x 1024 the polar rows' halos (117 columns each side) leave 86-column tiles; at
# 1024 x 1440 they (163) leave fewer than 32 owned columns, so that handle runs the per-point
# adjoint kernels.  Advection (halo max(M, Mv, nv of the row to the north)): 731 x 8 and 96 x 24 fit
# 256 threads in every row; at 512 x 1024 four rows next to the poles (halos up to 255) and at
# 1024 x 1440 five (up to 511) go with the pole rows through the per-point kernels.
@pytest.mark.parametrize("nx,ny,nz", [(731, 8, 3), (96, 24, 4), (512, 1024, 2), (1024, 1440, 1)])
@pytest.mark.parametrize("process", ["A", "L"])
def test_stage_adjoint_fp64_tile_forms(nx, ny, nz, process):
    """The stage adjoint equals the oracle for each tiling of the rows."""
    print(f"stage adjoint fp64 {process} {nx}x{ny}x{nz}", flush=True)
    cfg = small(nx, ny, nz)
    st = synth.make_state(cfg)
    ao = synth.random_like(st, 31)
    ch = 200.0
    wb, wi = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"]).adj_stage(st, ao, ch, process)
    core = _core(cfg, st, "fp64")
    d = core.to_device(st)
    a = core.to_device(ao)
    ab = {k: torch.zeros_like(v) for k, v in d.items()}
    ai = {k: torch.zeros_like(v) for k, v in d.items()}
    core.stage_adjoint(process, ch, d, a, ab, ai)
    gb, gi = _host(ab), _host(ai)
    for k in ("U", "V", "Phi", "ps"):
        assert _rel(gb[k], wb[k]) < 1e-12, ("base", k)
        assert _rel(gi[k], wi[k]) < 1e-12, ("in", k)


@pytest.mark.parametrize("process", ["A", "L"])
def test_stage_adjoint_aliased_buffers(process):
    """With the base and input adjoints in one buffer, the result is the sum of both parts."""
    cfg = small(64, 32, 4)
    st = synth.make_state(cfg)
    ao = synth.random_like(st, 32)
    ch = 150.0
    wb, wi = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"]).adj_stage(st, ao, ch, process)
    core = _core(cfg, st, "fp64")
    d = core.to_device(st)
    a = core.to_device(ao)
    acc = {k: torch.zeros_like(v) for k, v in d.items()}
    core.stage_adjoint(process, ch, d, a, acc, acc)
    got = _host(acc)
    for k in ("U", "V", "Phi", "ps"):
        want = wb[k] + wi[k]
        assert _rel(got[k], want) < 1e-12, (k, _rel(got[k], want))


def test_single_level():
    """nz = 1: a step and the step adjoint equal the oracle."""
    cfg = small(64, 32, 1)
    st = synth.make_state(cfg)
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"])
    core = _core(cfg, st, "fp64")
    d = core.to_device(st)
    core.step(d, 2)
    want = o.step(st, 2, cfg.dt)
    got = _host(d)
    for k in ("U", "V", "Phi", "ps"):
        assert _rel(got[k], want[k]) < 1e-11, (k, _rel(got[k], want[k]))
    lam0 = synth.random_like(st, 33)
    wl = o.adj_step(st, lam0, cfg.dt)
    lam = core.to_device(lam0)
    core.step_adjoint(core.to_device(st), lam)
    gl = _host(lam)
    for k in ("U", "V", "Phi", "ps"):
        assert _rel(gl[k], wl[k]) < 1e-11, (k, _rel(gl[k], wl[k]))


def test_zero_steps_is_identity():
    cfg = small(40, 20, 3)
    st = synth.make_state(cfg)
    core = _core(cfg, st, "fp32", forward_only=True)
    d = core.to_device(st)
    ref = {k: v.clone() for k, v in d.items()}
    core.step(d, 0)
    torch.cuda.synchronize()
    for k in d:
        assert torch.equal(d[k], ref[k]), k


@pytest.mark.parametrize("process", ["A", "L"])
def test_longest_rows_fp32(process):
    """Rows of 4096 columns (the largest accepted) run in zonal tiles like any other and equal the
    oracle's stage."""
    cfg = small(4096, 8, 2)
    st = synth.make_state(cfg)
    st32 = {k: st[k].astype(np.float32).astype(np.float64) for k in ("U", "V", "Phi", "ps")}
    ch = 60.0
    want = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"]).stage(st32, st32, ch, process)
    core = _core(cfg, st, "fp32", forward_only=True)
    d = core.to_device(st32)
    out = {k: torch.empty_like(v) for k, v in d.items()}
    got = _host(core.stage(process, ch, d, d, out))
    for k in ("U", "V", "Phi", "ps"):
        inc = want[k] - st32[k]
        scale = max(np.abs(inc).max(), np.abs(want[k]).max() * 1e-7)
        err = np.abs(got[k] - want[k]).max() / scale
        assert err < 2e-3, (k, err)


def test_refused_sizes():
    """Rows above 4096 columns, grids below the minimum and too many levels are argument errors,
    reported at create (not at the first step)."""
    from paper_2103_10114_amd import Dycore, DycoreError
    with pytest.raises(DycoreError):
        Dycore(4097, 8, 3, 60.0, prec="fp32", forward_only=True)
    with pytest.raises(DycoreError):
        Dycore(7, 8, 3, 60.0, prec="fp64", forward_only=True)
    with pytest.raises(DycoreError):
        Dycore(64, 8, 129, 60.0, prec="fp64", forward_only=True)


@pytest.mark.parametrize("process", ["A", "L"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stage_adjoint_adds_to_nonzero_accumulators(process, prec):
    """The stage adjoint adds into accumulators that already hold values (on a grid where the
    adaptation adjoint runs row-fused): FP64 totals equal initial values + the oracle's
    contributions to 1e-12; FP32 increments equal the contributions to 1e-3 relative L2 (as the FP32
    step adjoint).  An overwrite would miss by the size of the initial values."""
    print(f"stage adjoint += {prec} {process}", flush=True)
    cfg = small(96, 24, 4)
    st = synth.make_state(cfg)
    if prec == "fp32":
        st = dict(st, **{k: st[k].astype(np.float32).astype(np.float64) for k in ("U", "V", "Phi", "ps")})
    ao = synth.random_like(st, 34)
    ch = 120.0
    wb, wi = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"]).adj_stage(st, ao, ch, process)
    core = _core(cfg, st, prec)
    d = core.to_device(st)
    a = core.to_device(ao)
    ab = core.to_device(synth.random_like(st, 35))
    ai = core.to_device(synth.random_like(st, 36))
    b0, i0 = _host(ab), _host(ai)
    core.stage_adjoint(process, ch, d, a, ab, ai)
    gb, gi = _host(ab), _host(ai)
    for k in ("U", "V", "Phi", "ps"):
        for tag, got, start, want in (("base", gb, b0, wb), ("in", gi, i0, wi)):
            inc = got[k] - start[k]
            if prec == "fp64":
                err = _rel(got[k], start[k] + want[k])
                assert err < 1e-12, (tag, k, err)
            else:
                nw = np.linalg.norm(want[k])
                err = np.linalg.norm(inc - want[k]) / max(nw, 1e-30)
                assert err < 1e-3 or np.linalg.norm(inc - want[k]) < 1e-5 * np.linalg.norm(start[k]), (tag, k, err)
