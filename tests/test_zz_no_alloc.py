"""The no-allocation diagnostics entry point (static device scratch) against dycore_diagnostics,
through the C-ABI: two calls in a row, the second on a smaller grid, in both precisions."""
import dataclasses

import numpy as np
import pytest

from paper_2103_10114_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _case(cfg, prec):
    from paper_2103_10114_amd import Dycore
    st = synth.make_state(cfg)
    core = Dycore(cfg.nx, cfg.ny, cfg.nz, cfg.dt, prec=prec, phis=st["phis"], forward_only=True)
    return core, core.to_device(st)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_diagnostics_matches(prec):
    big = synth.CONFIGS["c2"]
    small = dataclasses.replace(synth.CONFIGS["c1"], nx=64, ny=32, nz=5, degree=5, seed=9)
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    for cfg in (big, small):            # the second call reuses the array with fewer rows
        print(f"noalloc diagnostics {prec} {cfg.nx}x{cfg.ny}x{cfg.nz}", flush=True)
        core, d = _case(cfg, prec)
        core.step(d, 1)
        core.diagnostics_noalloc(d, out)
        torch.cuda.synchronize()
        m, e = core.diagnostics(d)
        got = out.cpu().numpy()
        assert np.isfinite(got).all()
        assert got[0] == m and got[1] == e, (got, m, e)


def test_noalloc_diagnostics_row_limit():
    """More than 4097 rows do not fit the static array: an argument error, nothing enqueued."""
    from paper_2103_10114_amd import Dycore, DycoreError
    core = Dycore(8, 4100, 1, 60.0, prec="fp64", forward_only=True)
    st = core.empty_state()
    st["ps"].fill_(1e5)
    out = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
    with pytest.raises(DycoreError):
        core.diagnostics_noalloc(st, out)
    torch.cuda.synchronize()
    assert out.cpu().tolist() == [-1.0, -1.0]
