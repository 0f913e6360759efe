"""Python binding of the CGP C ABI with torch tensors as device memory.

The functions carry the C names (cgp_create, cgp_step, cgp_adjoint_step, ...)
and only marshal arguments: tensor -> device pointer, torch stream -> HIP
stream, shapes and dtypes checked against the handle.  ``Basin`` and
``Ensemble`` own a workspace tensor and a handle; ``Trajectory`` is the
``torch.autograd.Function`` of an nsteps CGPRK3 trajectory whose backward
runs the library's adjoint over checkpointed segments.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import CGP_F32, CGP_F64, CGPError, call, cgp_config, cgp_launch  # noqa: F401

_TORCH_DTYPE = {CGP_F32: torch.float32, CGP_F64: torch.float64}


def make_config(nx, ny, level=0, nlayers=1, dtype="f64", lx=1.0, ly=2.0, y0=-1.0,
                inv_re=1.0, inv_ro=0.0, f1=0.0, f2=0.0, drag=0.0, dt=1e-4,
                cfl=0.0, solver=0, mg_cycles=0, fused_rows=0) -> cgp_config:
    dt_code = {"f64": CGP_F64, "f32": CGP_F32}.get(dtype, dtype)  # ints pass through
    return cgp_config(nx=nx, ny=ny, level=level, nlayers=nlayers, dtype=dt_code, reserved=0,
                      lx=lx, ly=ly, y0=y0, inv_re=inv_re, inv_ro=inv_ro, f1=f1, f2=f2,
                      drag=drag, dt=dt, cfl=cfl, solver=solver, mg_cycles=mg_cycles,
                      fused_rows=fused_rows)


def with_fused_rows(cfgs, rows: int) -> list:
    """Copies of cfgs with cgp_config.fused_rows = rows (the autotuner's
    choice for a workload)."""
    out = []
    for c in cfgs:
        d = cgp_config.from_buffer_copy(c)
        d.fused_rows = rows
        out.append(d)
    return out


def config_from_case(case, dtype: Optional[str] = None) -> cgp_config:
    """cgp_config of a cgp_inputs.Case."""
    return make_config(case.nx, case.ny, case.level, case.nlayers, dtype or case.dtype, case.lx,
                       case.ly, case.y0, case.inv_re, case.inv_ro, case.f1, case.f2, case.drag,
                       case.dt, case.cfl, case.solver, case.mg_cycles)


def stream_ptr(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_tensor(t, dtype, numel, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise CGPError(_lib.CGP_ERR_INVALID, f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise CGPError(_lib.CGP_ERR_INVALID, f"{name} must be contiguous")
    if t.dtype != dtype:
        raise CGPError(_lib.CGP_ERR_INVALID, f"{name} has dtype {t.dtype}, handle uses {dtype}")
    if numel is not None and t.numel() != numel:
        raise CGPError(_lib.CGP_ERR_INVALID, f"{name} has {t.numel()} elements, expected {numel}")


# ----------------------------------------------------------------------------- C names
def cgp_workspace_size(cfg: cgp_config) -> int:
    n = ctypes.c_size_t()
    call("cgp_workspace_size", ctypes.byref(cfg), ctypes.byref(n))
    return n.value


def cgp_create(cfg: cgp_config, workspace: torch.Tensor, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    call("cgp_create", ctypes.byref(cfg), _ptr(workspace), workspace.numel(),
         ctypes.c_void_p(stream_ptr(stream)), ctypes.byref(h))
    return h


def cgp_destroy(h):
    call("cgp_destroy", h)


def cgp_step(h, omega, forcing, psi_out=None, nsteps=1, stream=None):
    call("cgp_step", h, _ptr(omega), _ptr(forcing), _ptr(psi_out), int(nsteps),
         ctypes.c_void_p(stream_ptr(stream)))


def cgp_step_noalloc(cfg: cgp_config, omega, forcing, psi_out=None, nsteps=1, stream=None):
    """cgp_step of a fresh handle whose workspace is the library's static device
    scratch (no device allocation by the library or by this binding)."""
    call("cgp_step_noalloc", ctypes.byref(cfg), _ptr(omega), _ptr(forcing), _ptr(psi_out),
         int(nsteps), ctypes.c_void_p(stream_ptr(stream)))


def cgp_time_state(h, out, stream=None):
    """out (FP64 device tensor, 2 per member) <- (dt of the latest step, model time)."""
    call("cgp_time_state", h, _ptr(out), ctypes.c_void_p(stream_ptr(stream)))


def cgp_step_mean(h, omega, forcing, nsteps, total, use_graph=True, stream=None):
    call("cgp_step_mean", h, _ptr(omega), _ptr(forcing), int(nsteps), _ptr(total),
         int(bool(use_graph)), ctypes.c_void_p(stream_ptr(stream)))


def cgp_accumulate(h, field, total, weight=1.0, times_dt=False, stream=None):
    """total (FP64 device tensor, the handle's field layout) += weight [* dt] * field."""
    call("cgp_accumulate", h, _ptr(field), _ptr(total), float(weight), int(bool(times_dt)),
         ctypes.c_void_p(stream_ptr(stream)))


def cgp_solve(h, omega, psi, stream=None):
    call("cgp_solve", h, _ptr(omega), _ptr(psi), ctypes.c_void_p(stream_ptr(stream)))


def cgp_diagnostics(h, omega, psi, out, stream=None):
    call("cgp_diagnostics", h, _ptr(omega), _ptr(psi), _ptr(out),
         ctypes.c_void_p(stream_ptr(stream)))


def cgp_check_finite(h, field, flag, stream=None):
    call("cgp_check_finite", h, _ptr(field), field.numel(), _ptr(flag),
         ctypes.c_void_p(stream_ptr(stream)))


def cgp_assert_finite(h, field, stream=None):
    """Raises CGPError (CGP_ERR_NONFINITE) if field holds a NaN or an infinity."""
    call("cgp_assert_finite", h, _ptr(field), field.numel(), ctypes.c_void_p(stream_ptr(stream)))


def cgp_tape_size(cfg: cgp_config, nsteps: int) -> int:
    n = ctypes.c_size_t()
    call("cgp_tape_size", ctypes.byref(cfg), int(nsteps), ctypes.byref(n))
    return n.value


def cgp_adjoint_step(h, omega_n, forcing, nsteps, lam, grad_forcing, tape, stream=None):
    call("cgp_adjoint_step", h, _ptr(omega_n), _ptr(forcing), int(nsteps), _ptr(lam),
         _ptr(grad_forcing), _ptr(tape), tape.numel() * tape.element_size(),
         ctypes.c_void_p(stream_ptr(stream)))


def _cfg_array(cfgs: Sequence[cgp_config]):
    arr = (cgp_config * len(cfgs))()
    for i, c in enumerate(cfgs):
        arr[i] = c
    return arr


def cgp_ensemble_offsets(cfgs: Sequence[cgp_config]):
    arr = _cfg_array(cfgs)
    offs = (ctypes.c_int64 * len(cfgs))()
    tot = ctypes.c_int64()
    call("cgp_ensemble_offsets", arr, len(cfgs), offs, ctypes.byref(tot))
    return list(offs), tot.value


def cgp_ensemble_workspace_size(cfgs: Sequence[cgp_config]) -> int:
    arr = _cfg_array(cfgs)
    n = ctypes.c_size_t()
    call("cgp_ensemble_workspace_size", arr, len(cfgs), ctypes.byref(n))
    return n.value


def cgp_ensemble_create(cfgs: Sequence[cgp_config], workspace: torch.Tensor, stream=None):
    arr = _cfg_array(cfgs)
    h = ctypes.c_void_p()
    call("cgp_ensemble_create", arr, len(cfgs), _ptr(workspace), workspace.numel(),
         ctypes.c_void_p(stream_ptr(stream)), ctypes.byref(h))
    return h


def cgp_ensemble_step(h, omega_packed, forcing_packed, nsteps=1, use_graph=True, stream=None):
    call("cgp_ensemble_step", h, _ptr(omega_packed), _ptr(forcing_packed), int(nsteps),
         1 if use_graph else 0, ctypes.c_void_p(stream_ptr(stream)))


def cgp_time_passes(h, omega, forcing, reps, stream=None):
    """Mean ms per launch of passes A, B, C, D, the fused C + D pass and the
    fused pass with the next stage's pass A (0 for the last two when the handle
    has none); reps back-to-back launches each; synchronises."""
    ms = (ctypes.c_double * 6)()
    call("cgp_time_passes", h, _ptr(omega), _ptr(forcing), int(reps), ms,
         ctypes.c_void_p(stream_ptr(stream)))
    return list(ms)


def cgp_set_launch(h, mode=0, b_tile=1, f_tile=1, wg_per_cu=0, stream=None):
    """Launch mode of the handle's steps: 0 per-pass launches, 1 one persistent
    launch per RK3 stage (tiles of b_tile pass-B and f_tile fused blocks)."""
    lc = cgp_launch(mode=mode, b_tile=b_tile, f_tile=f_tile, wg_per_cu=wg_per_cu)
    call("cgp_set_launch", h, ctypes.byref(lc), ctypes.c_void_p(stream_ptr(stream)))


def cgp_get_launch(h):
    """(dict of the launch setting, whether the persistent mode is available)."""
    lc = cgp_launch()
    avail = ctypes.c_int32()
    call("cgp_get_launch", h, ctypes.byref(lc), ctypes.byref(avail))
    return dict(mode=lc.mode, b_tile=lc.b_tile, f_tile=lc.f_tile,
                wg_per_cu=lc.wg_per_cu), bool(avail.value)


def cgp_persistent_fault(h, stream=None) -> int:
    flag = ctypes.c_int32()
    call("cgp_persistent_fault", h, ctypes.byref(flag), ctypes.c_void_p(stream_ptr(stream)))
    return flag.value


def cgp_time_step_passes(h, omega, forcing, nsteps, stream=None):
    """nsteps time steps (direct launches) with HIP events around every pass B
    and fused-pass launch: mean ms per launch of each and mean ms per step."""
    ms = (ctypes.c_double * 3)()
    call("cgp_time_step_passes", h, _ptr(omega), _ptr(forcing), int(nsteps), ms,
         ctypes.c_void_p(stream_ptr(stream)))
    return list(ms)


def cgp_last_error() -> str:
    return _lib.load().cgp_last_error().decode(errors="replace")


def cgp_version() -> str:
    return _lib.load().cgp_version().decode()


# ----------------------------------------------------------------------------- owners
class Basin:
    """One basin: workspace tensor + handle.  Fields are torch tensors of shape
    (ny+1, nx+1) or (2, ny+1, nx+1) on the handle's device and dtype."""

    def __init__(self, cfg: cgp_config, device="cuda", stream=None):
        self.cfg = cfg
        self.device = torch.device(device)
        self.dtype = _TORCH_DTYPE[cfg.dtype]
        self.shape = ((cfg.ny + 1, cfg.nx + 1) if cfg.nlayers == 1
                      else (2, cfg.ny + 1, cfg.nx + 1))
        self.numel = cfg.nlayers * (cfg.ny + 1) * (cfg.nx + 1)
        nbytes = cgp_workspace_size(cfg)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.handle = cgp_create(cfg, self.workspace, stream)

    def _chk(self, t, name, numel=None):
        _check_tensor(t, self.dtype, self.numel if numel is None else numel, name)

    def step(self, omega, forcing, nsteps=1, psi_out=None, stream=None):
        self._chk(omega, "omega")
        self._chk(forcing, "forcing", (self.cfg.ny + 1) * (self.cfg.nx + 1))
        if psi_out is not None:
            self._chk(psi_out, "psi_out")
        cgp_step(self.handle, omega, forcing, psi_out, nsteps, stream)
        return omega

    def solve(self, omega, psi=None, stream=None):
        self._chk(omega, "omega")
        psi = torch.empty_like(omega) if psi is None else psi
        self._chk(psi, "psi")
        cgp_solve(self.handle, omega, psi, stream)
        return psi

    def diagnostics(self, omega, psi, out=None, stream=None):
        self._chk(omega, "omega")
        self._chk(psi, "psi")
        out = torch.empty(2 * self.cfg.nlayers, dtype=torch.float64, device=self.device) \
            if out is None else out
        cgp_diagnostics(self.handle, omega, psi, out, stream)
        return out

    def check_finite(self, field, stream=None):
        _check_tensor(field, self.dtype, None, "field")
        flag = torch.empty(1, dtype=torch.int32, device=self.device)
        cgp_check_finite(self.handle, field, flag, stream)
        return flag

    def assert_finite(self, field, stream=None):
        _check_tensor(field, self.dtype, None, "field")
        cgp_assert_finite(self.handle, field, stream)

    def time_state(self, stream=None):
        """FP64 device tensor [dt of the latest step, model time advanced]."""
        out = torch.empty(2, dtype=torch.float64, device=self.device)
        cgp_time_state(self.handle, out, stream)
        return out

    def step_mean(self, omega, forcing, nsteps, total, use_graph=True, stream=None):
        """nsteps steps; after each, total (FP64, the field's shape) += dt * omega."""
        self._chk(omega, "omega")
        self._chk(forcing, "forcing", (self.cfg.ny + 1) * (self.cfg.nx + 1))
        if total.dtype != torch.float64 or total.numel() != self.numel or not total.is_cuda:
            raise CGPError(_lib.CGP_ERR_INVALID, "total must be an FP64 device tensor of the field")
        cgp_step_mean(self.handle, omega, forcing, nsteps, total, use_graph, stream)
        return omega

    def accumulate(self, field, total, weight=1.0, times_dt=False, stream=None):
        """total (FP64, the field's shape) += weight [* dt of the latest step] * field."""
        self._chk(field, "field")
        if total.dtype != torch.float64 or total.numel() != self.numel or not total.is_cuda:
            raise CGPError(_lib.CGP_ERR_INVALID, "total must be an FP64 device tensor of the field")
        cgp_accumulate(self.handle, field, total, weight, times_dt, stream)
        return total

    def tape(self, nsteps):
        n = cgp_tape_size(self.cfg, nsteps)
        return torch.empty(n // 8, dtype=torch.float64, device=self.device)

    def adjoint_step(self, omega_n, forcing, nsteps, lam, grad_forcing, tape=None, stream=None):
        tape = self.tape(nsteps) if tape is None else tape
        for t, nm in ((omega_n, "omega_n"), (forcing, "forcing"), (lam, "lambda"),
                      (grad_forcing, "grad_forcing")):
            self._chk(t, nm)
        cgp_adjoint_step(self.handle, omega_n, forcing, nsteps, lam, grad_forcing, tape, stream)
        return lam, grad_forcing

    def close(self):
        if self.handle is not None:
            cgp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ensemble:
    """Members packed back to back; one launch per pass over all members."""

    def __init__(self, cfgs: List[cgp_config], device="cuda", stream=None):
        self.cfgs = list(cfgs)
        self.device = torch.device(device)
        self.dtype = _TORCH_DTYPE[self.cfgs[0].dtype]
        self.offsets, self.total = cgp_ensemble_offsets(self.cfgs)
        nbytes = cgp_ensemble_workspace_size(self.cfgs)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.handle = cgp_ensemble_create(self.cfgs, self.workspace, stream)

    def member_view(self, packed, m):
        c = self.cfgs[m]
        n = c.nlayers * (c.ny + 1) * (c.nx + 1)
        shape = (c.ny + 1, c.nx + 1) if c.nlayers == 1 else (2, c.ny + 1, c.nx + 1)
        return packed[self.offsets[m]: self.offsets[m] + n].view(shape)

    def pack(self, fields):
        out = torch.empty(self.total, dtype=self.dtype, device=self.device)
        for m, f in enumerate(fields):
            self.member_view(out, m).copy_(torch.as_tensor(f))
        return out

    def step(self, omega_packed, forcing_packed, nsteps=1, use_graph=True, stream=None):
        _check_tensor(omega_packed, self.dtype, self.total, "omega_packed")
        _check_tensor(forcing_packed, self.dtype, self.total, "forcing_packed")
        cgp_ensemble_step(self.handle, omega_packed, forcing_packed, nsteps, use_graph, stream)
        return omega_packed

    def set_launch(self, mode=0, b_tile=1, f_tile=1, wg_per_cu=0, stream=None):
        cgp_set_launch(self.handle, mode, b_tile, f_tile, wg_per_cu, stream)

    def launch(self):
        return cgp_get_launch(self.handle)

    def persistent_fault(self, stream=None) -> int:
        return cgp_persistent_fault(self.handle, stream)

    def time_state(self, stream=None):
        """FP64 device tensor (members, 2): dt of each member's latest step and
        its model time advanced."""
        out = torch.empty((len(self.cfgs), 2), dtype=torch.float64, device=self.device)
        cgp_time_state(self.handle, out, stream)
        return out

    def close(self):
        if self.handle is not None:
            cgp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Trajectory(torch.autograd.Function):
    """omega_T = Phi^nsteps(omega_0; F) with checkpoints every `ckpt_every` steps.

    backward returns dL/domega_0 and dL/dF from the library adjoint, segment by
    segment in reverse, each segment recomputed from its checkpoint."""

    @staticmethod
    def forward(ctx, omega0, forcing, basin: Basin, nsteps: int, ckpt_every: int):
        w = omega0.detach().clone()
        F = forcing.detach().contiguous()
        ckpts = []
        done = 0
        while done < nsteps:
            k = min(ckpt_every, nsteps - done)
            ckpts.append((w.clone(), k))
            basin.step(w, F, nsteps=k)
            done += k
        ctx.basin = basin
        ctx.ckpts = ckpts
        ctx.save_for_backward(F)
        return w

    @staticmethod
    def backward(ctx, grad_out):
        (F,) = ctx.saved_tensors
        basin = ctx.basin
        lam = grad_out.detach().clone().contiguous()
        gF = torch.zeros_like(F)
        kmax = max(k for _, k in ctx.ckpts)
        tape = basin.tape(kmax)
        for w0, k in reversed(ctx.ckpts):
            basin.adjoint_step(w0, F, k, lam, gF, tape)
        return lam, gF, None, None, None
