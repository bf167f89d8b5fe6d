"""MI355X leap-format dynamical-core step: Python binding of libdycore.

Argument marshalling only: every step of the computation runs in the HIP
kernels of libdycore.so (built in-tree by `paper_2103_10114_amd.build`).
PyTorch supplies device memory and the current stream.  There is no CPU
fallback: a missing library raises.

Fields are torch tensors on the GPU, contiguous, float32 or float64:
  U (ny+1, nz, nx), V (ny, nz, nx), Phi (ny+1, nz, nx), ps (ny+1, nx)
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdycore.so")
_lib = None

DYCORE_FP32, DYCORE_FP64 = 0, 1
DYCORE_FORWARD_ONLY = 1
DYCORE_LOWLAT_FILTERS = 2
DYCORE_SINGLE_STREAM = 4
KEYS = ("U", "V", "Phi", "ps")


class DycoreError(RuntimeError):
    pass


class _Config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("dt", ctypes.c_double),
                ("n_adapt_substeps", ctypes.c_int), ("prec", ctypes.c_int),
                ("sigma_half", ctypes.POINTER(ctypes.c_double)), ("phis", ctypes.POINTER(ctypes.c_double)),
                ("a", ctypes.c_double), ("omega", ctypes.c_double), ("g", ctypes.c_double),
                ("rd", ctypes.c_double), ("cp", ctypes.c_double), ("p0", ctypes.c_double), ("t0", ctypes.c_double),
                ("flags", ctypes.c_uint), ("block", ctypes.c_int), ("kappa_star", ctypes.c_double)]


def lib():
    """Load libdycore.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DycoreError(f"{LIB_PATH} is missing: build it with python -m paper_2103_10114_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.dycore_create.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(vp)]
        L.dycore_destroy.argtypes = [vp]
        L.dycore_step.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int, vp]
        L.dycore_stage.argtypes = [vp, ctypes.c_int, ctypes.c_double] + [vp] * 12 + [vp]
        L.dycore_process_run.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_double] + [vp] * 4 + [vp]
        L.dycore_step_adjoint.argtypes = [vp] + [vp] * 8 + [vp]
        L.dycore_step_record.argtypes = [vp] + [vp] * 4 + [vp]
        L.dycore_step_adjoint_recorded.argtypes = [vp] + [vp] * 4 + [vp]
        L.dycore_stage_adjoint.argtypes = [vp, ctypes.c_int, ctypes.c_double] + [vp] * 16 + [vp]
        L.dycore_diagnostics.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double), vp]
        L.dycore_diagnostics_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.dycore_check_finite.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_longlong), vp]
        L.dycore_leap_table.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.dycore_substeps.argtypes = [vp]
        L.dycore_block.argtypes = [vp]
        L.dycore_workspace_bytes.argtypes = [vp]
        L.dycore_kernel_timer_start.argtypes = [vp, ctypes.c_int]
        L.dycore_kernel_timer_stop.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
        L.dycore_workspace_bytes.restype = ctypes.c_size_t
        L.dycore_strerror.argtypes = [ctypes.c_int]
        L.dycore_strerror.restype = ctypes.c_char_p
        L.dycore_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)] + [ctypes.POINTER(vp)] * 4 + \
            [ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]
        L.dycore_batch_step.argtypes = [vp, ctypes.c_int, vp]
        L.dycore_batch_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise DycoreError(f"libdycore: {lib().dycore_strerror(rc).decode()} ({rc})")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None):
    import torch
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("fields must be contiguous GPU tensors")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


class Dycore:
    """One grid (nx longitudes, ny latitude intervals, nz levels) and time step dt."""

    def __init__(self, nx, ny, nz, dt, prec="fp32", phis=None, msub=0, block=0, forward_only=False,
                 sigma_half=None, filters=False, kappa_star=0.0, single_stream=False):
        import numpy as np
        import torch
        self.nx, self.ny, self.nz, self.dt = nx, ny, nz, float(dt)
        self.prec = prec
        self.dtype = torch.float32 if prec == "fp32" else torch.float64
        c = _Config()
        c.nx, c.ny, c.nz, c.dt = nx, ny, nz, float(dt)
        c.n_adapt_substeps = int(msub)
        c.prec = DYCORE_FP32 if prec == "fp32" else DYCORE_FP64
        self._phis = None if phis is None else np.ascontiguousarray(phis, dtype=np.float64)
        self._sig = None if sigma_half is None else np.ascontiguousarray(sigma_half, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        c.phis = self._phis.ctypes.data_as(dp) if self._phis is not None else None
        c.sigma_half = self._sig.ctypes.data_as(dp) if self._sig is not None else None
        c.flags = ((DYCORE_FORWARD_ONLY if forward_only else 0) | (DYCORE_LOWLAT_FILTERS if filters else 0) |
                   (DYCORE_SINGLE_STREAM if single_stream else 0))
        c.block = int(block)
        c.kappa_star = float(kappa_star)
        h = ctypes.c_void_p()
        _check(lib().dycore_create(ctypes.byref(c), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().dycore_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- shapes / allocation
    def shapes(self):
        nx, ny, nz = self.nx, self.ny, self.nz
        return {"U": (ny + 1, nz, nx), "V": (ny, nz, nx), "Phi": (ny + 1, nz, nx), "ps": (ny + 1, nx)}

    def empty_state(self):
        import torch
        return {k: torch.zeros(s, dtype=self.dtype, device="cuda") for k, s in self.shapes().items()}

    def to_device(self, st):
        import torch
        return {k: torch.as_tensor(st[k]).to(device="cuda", dtype=self.dtype).contiguous() for k in KEYS}

    def _p(self, st):
        return [_ptr(st[k], self.dtype) for k in KEYS]

    # -- calls
    @property
    def substeps(self):
        return int(lib().dycore_substeps(self.h))

    @property
    def block(self):
        return int(lib().dycore_block(self.h))

    def workspace_bytes(self):
        return int(lib().dycore_workspace_bytes(self.h))

    def leap_table(self):
        import numpy as np
        m = np.zeros(self.ny + 1, dtype=np.int32)
        mv = np.zeros(self.ny, dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int)
        _check(lib().dycore_leap_table(self.h, m.ctypes.data_as(ip), mv.ctypes.data_as(ip)))
        return m, mv

    def step(self, st, nsteps=1):
        """Advance the fields of st in place by nsteps outer steps."""
        _check(lib().dycore_step(self.h, *self._p(st), int(nsteps), _stream()))
        return st

    def process_run(self, st, process, n_rk, hstep):
        """n_rk RK3 steps of one process alone, in place (same stage kernels as step)."""
        proc = 0 if process in (0, "A") else 1
        _check(lib().dycore_process_run(self.h, proc, int(n_rk), float(hstep), *self._p(st), _stream()))
        return st

    def stage(self, process, ch, base, inp, out):
        proc = 0 if process in (0, "A") else 1
        _check(lib().dycore_stage(self.h, proc, float(ch), *self._p(base), *self._p(inp), *self._p(out), _stream()))
        return out

    def tendency(self, inp, process):
        """T(in) as a stage with zero base and ch = 1."""
        base = {k: v.new_zeros(v.shape) for k, v in inp.items() if k in KEYS}
        out = {k: v.new_zeros(v.shape) for k, v in inp.items() if k in KEYS}
        return self.stage(process, 1.0, base, inp, out)

    def step_adjoint(self, st0, adj):
        """adj (adjoint of the step output) is replaced in place by the adjoint of the step input."""
        _check(lib().dycore_step_adjoint(self.h, *self._p(st0), *self._p(adj), _stream()))
        return adj

    def step_record(self, st):
        """One outer step in place (as step(st, 1)) that keeps its stage inputs for step_adjoint_recorded."""
        _check(lib().dycore_step_record(self.h, *self._p(st), _stream()))
        return st

    def step_adjoint_recorded(self, adj):
        """Adjoint of the step last taken with step_record; adj is replaced in place as in step_adjoint."""
        _check(lib().dycore_step_adjoint_recorded(self.h, *self._p(adj), _stream()))
        return adj

    def kernel_timer_start(self, max_launches):
        """Arm live HIP-event timing of the row-fused adaptation-stage adjoint kernel's launches."""
        _check(lib().dycore_kernel_timer_start(self.h, int(max_launches)))

    def kernel_timer_stop(self):
        """(total ms, launches) of the launches timed since kernel_timer_start; disarms."""
        ms, n = ctypes.c_double(), ctypes.c_int()
        _check(lib().dycore_kernel_timer_stop(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def stage_adjoint(self, process, ch, inp, aout, abase, ain):
        proc = 0 if process in (0, "A") else 1
        _check(lib().dycore_stage_adjoint(self.h, proc, float(ch), *self._p(inp), *self._p(aout),
                                          *self._p(abase), *self._p(ain), _stream()))

    def diagnostics(self, st):
        m = ctypes.c_double()
        e = ctypes.c_double()
        _check(lib().dycore_diagnostics(self.h, *self._p(st), ctypes.byref(m), ctypes.byref(e), _stream()))
        return m.value, e.value

    def diagnostics_noalloc(self, st, out):
        """Mass and energy into out (a float64 GPU tensor of 2 entries), with no allocation and no
        host synchronisation."""
        _check(lib().dycore_diagnostics_noalloc(self.h, *self._p(st), _ptr(out), _stream()))
        return out

    def count_nonfinite(self, st):
        c = ctypes.c_longlong()
        rc = lib().dycore_check_finite(self.h, *self._p(st), ctypes.byref(c), _stream())
        if rc not in (0, -4):
            _check(rc)
        return int(c.value)


class Batch:
    """Ensemble members advanced together, one persistent launch per stage."""

    def __init__(self, cores, states, block=0, grid=0):
        self.cores = list(cores)
        self.states = list(states)
        n = len(self.cores)
        vp = ctypes.c_void_p
        hs = (vp * n)(*[c.h.value for c in self.cores])
        arrs = []
        for k in KEYS:
            arrs.append((vp * n)(*[_ptr(s[k], c.dtype).value for c, s in zip(self.cores, self.states)]))
        b = vp()
        _check(lib().dycore_batch_create(n, hs, *arrs, int(block), int(grid), ctypes.byref(b)))
        self.b = b

    def step(self, nsteps=1):
        _check(lib().dycore_batch_step(self.b, int(nsteps), _stream()))

    @classmethod
    def autotune(cls, cores, states, blocks=(128, 256, 384, 512), steps=2):
        """Time the batched step at each workgroup size in `blocks` (on copies of the states, so the
        members are not advanced) and return (Batch at the fastest size, {block: ms per step}).
        Sizes the batch cannot use (tiles that do not fit, above the register budget's 512 threads)
        are skipped.  Results do not depend on the workgroup size, so tuning changes speed only."""
        import torch
        copies = [_clone(st) for st in states]
        table = {}
        for blk in blocks:
            try:
                b = cls(cores, copies, block=blk)
            except DycoreError:
                continue
            b.step(1)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            b.step(steps)
            e1.record()
            e1.synchronize()
            table[blk] = e0.elapsed_time(e1) / steps
            b.close()
        del copies
        if not table:
            raise DycoreError("no workgroup size fits this batch")
        best = min(table, key=table.get)
        return cls(cores, states, block=best), table

    def close(self):
        if getattr(self, "b", None) is not None and self.b.value:
            lib().dycore_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------------------------
# autograd and multi-step adjoint windows
# ------------------------------------------------------------------------------------------------
def _clone(st):
    return {k: st[k].clone() for k in KEYS}


class _StepFn:
    """torch.autograd.Function for one outer step (built lazily so that importing the package does
    not import torch)."""
    _cls = None

    @classmethod
    def get(cls):
        if cls._cls is None:
            import torch

            class DycoreStep(torch.autograd.Function):
                @staticmethod
                def forward(ctx, core, U, V, Phi, ps):
                    st0 = {"U": U.detach().contiguous(), "V": V.detach().contiguous(),
                           "Phi": Phi.detach().contiguous(), "ps": ps.detach().contiguous()}
                    out = _clone(st0)
                    core.step(out, 1)
                    ctx.core = core
                    ctx.save_for_backward(st0["U"], st0["V"], st0["Phi"], st0["ps"])
                    return out["U"], out["V"], out["Phi"], out["ps"]

                @staticmethod
                def backward(ctx, gU, gV, gPhi, gps):
                    U, V, Phi, ps = ctx.saved_tensors
                    core = ctx.core
                    lam = {}
                    for k, gk, ref in (("U", gU, U), ("V", gV, V), ("Phi", gPhi, Phi), ("ps", gps, ps)):
                        lam[k] = (gk if gk is not None else torch.zeros_like(ref)).contiguous().clone()
                    core.step_adjoint({"U": U, "V": V, "Phi": Phi, "ps": ps}, lam)
                    return None, lam["U"], lam["V"], lam["Phi"], lam["ps"]

            cls._cls = DycoreStep
        return cls._cls


def dycore_step_fn(core, U, V, Phi, ps):
    """Differentiable outer step: returns (U, V, Phi, ps) after one step; backward runs the
    hand-written adjoint kernels."""
    return _StepFn.get().apply(core, U, V, Phi, ps)


def adjoint_window(core, state, nsteps, lam, ckpt_every=8, keep_trajectory=False):
    """Adjoint of nsteps outer steps starting at `state`: lam (adjoint of the final state) is
    replaced by the adjoint of the initial state.  Checkpoints are kept every ckpt_every steps;
    each window's step-start states are recomputed from its checkpoint in the reverse pass
    (keep_trajectory=True stores every step-start state instead).  Returns the final state and a
    dict with the checkpoint and window memory in bytes."""
    import torch
    nbytes = sum(state[k].numel() * state[k].element_size() for k in KEYS)
    y = _clone(state)
    ckpts = {}
    traj = {}
    for n in range(nsteps):
        if keep_trajectory:
            traj[n] = _clone(y)
        elif n % ckpt_every == 0:
            ckpts[n] = _clone(y)
        core.step(y, 1)
    final = y
    mem = {"state_bytes": nbytes, "checkpoints": len(ckpts), "checkpoint_bytes": len(ckpts) * nbytes,
           "window_bytes": 0 if keep_trajectory else min(ckpt_every, nsteps) * nbytes,
           "trajectory_bytes": len(traj) * nbytes}
    if keep_trajectory:
        for n in range(nsteps - 1, -1, -1):
            core.step_adjoint(traj[n], lam)
        return final, mem
    starts = sorted(ckpts)
    for w in reversed(starts):
        end = min(w + ckpt_every, nsteps)
        window = [_clone(ckpts[w])]
        for n in range(w, end - 1):
            nxt = _clone(window[-1])
            core.step(nxt, 1)
            window.append(nxt)
        for n in range(end - 1, w - 1, -1):
            core.step_adjoint(window[n - w], lam)
        del window
        torch.cuda.current_stream().synchronize()
    return final, mem
