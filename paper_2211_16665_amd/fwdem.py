"""ctypes binding of libfwdem.so (include/fwdem.h), argument marshalling only.

Every step of the modelling and adjoint path runs in the HIP library; this
module converts Python/NumPy/torch arguments to the C ABI, owns nothing but
torch tensors for device memory, and raises ``FwdError`` on a non-zero
status.  There is no CPU fallback: without the built library the import of
the product path fails.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, c_double, c_int, c_size_t, c_void_p,
                    byref)

import numpy as np
# torch first: libfwdem.so then binds the HIP runtime torch has loaded, so
# the library and the torch tensors it is handed share one runtime (loading
# the library first would bind the system runtime and torch a second one)
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libfwdem.so")

FWD_OK = 0
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OOM", 3: "HIP", 4: "NONFINITE", 5: "CFL",
          6: "BASIS", 7: "UNSUPPORTED", 8: "STATE"}
FWD_F32, FWD_F64 = 0, 1
FWD_ACC_F64, FWD_ACC_KAHAN, FWD_ACC_F32 = 0, 1, 2
FWD_MODE_FORWARD, FWD_MODE_ADJOINT = 0, 1
(FWD_TAB_WAVELET, FWD_TAB_NORM, FWD_TAB_OMEGA, FWD_TAB_CPML_X, FWD_TAB_CPML_Y,
 FWD_TAB_CPML_Z, FWD_TAB_BASIS, FWD_TAB_EDGE_SIGMA, FWD_TAB_METRIC_X, FWD_TAB_METRIC_Y,
 FWD_TAB_METRIC_Z) = range(11)
(FWD_OPT_GRAPH_STEPS, FWD_OPT_BLOCK_X, FWD_OPT_BLOCK_Y, FWD_OPT_XCD_REMAP,
 FWD_OPT_SAMPLE_EVERY, FWD_OPT_STRICT_CFL, FWD_OPT_DFT_BLOCK, FWD_OPT_VECTOR,
 FWD_OPT_SCHEDULE, FWD_OPT_ZCHUNK, FWD_OPT_TILE_ORDER, FWD_OPT_VECTOR_H,
 FWD_OPT_VTI_GRADIENT, FWD_OPT_FD_ORDER, FWD_OPT_LEAN, FWD_OPT_BARRIER_US,
 FWD_OPT_PERSIST_BLOCKS, FWD_OPT_BARRIER_SLEEP, FWD_OPT_DFT_DECIMATE,
 FWD_OPT_STREAM_STORES) = range(20)

FWD_STATIC_SCRATCH_BYTES = 32 << 20       # the static workspace of fwd_forward_static

ACC_MODES = {"f64": FWD_ACC_F64, "kahan": FWD_ACC_KAHAN, "f32": FWD_ACC_F32}
DTYPES = {"f32": FWD_F32, "f64": FWD_F64}


class FwdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fwdem {STATUS.get(status, status)}: {msg}")
        self.status = status


class fwd_plan_desc(Structure):
    _fields_ = [
        ("nx", c_int), ("ny", c_int), ("nz", c_int),
        ("x", POINTER(c_double)), ("y", POINTER(c_double)), ("z", POINTER(c_double)),
        ("npml", c_int),
        ("cpml_order", c_double), ("cpml_R", c_double), ("cpml_kappa_max", c_double),
        ("cpml_alpha_max", c_double), ("cpml_vref", c_double),
        ("f0", c_double),
        ("nfreq", c_int), ("freqs", POINTER(c_double)),
        ("nsrc", c_int), ("src_pos", POINTER(c_double)), ("src_mom", POINTER(c_double)),
        ("nrec", c_int), ("rec_pos", POINTER(c_double)),
        ("ncomp", c_int), ("rec_comp", POINTER(c_int)),
        ("field_dtype", c_int), ("acc_mode", c_int),
        ("rho_air_cap", c_double), ("cfl", c_double), ("dt", c_double), ("nt", c_int),
        ("src_kind", c_int),
    ]


class fwd_info(Structure):
    _fields_ = [
        ("dt", c_double), ("dt_cfl", c_double), ("nt", c_int),
        ("vmax", c_double), ("vref", c_double), ("tau", c_double), ("t0", c_double),
        ("src_scale", c_double),
        ("nx", c_int), ("ny", c_int), ("nz", c_int), ("px", c_int),
        ("n_rec_nodes", c_int), ("n_src_entries", c_int), ("n_adj_targets", c_int),
        ("have_basis", c_int), ("basis_iters", c_int),
        ("basis_gamma", c_double), ("basis_fit", c_double),
        ("workspace_bytes_forward", c_size_t), ("workspace_bytes_adjoint", c_size_t),
        ("volume_bytes", c_size_t), ("state_bytes", c_size_t),
    ]


# name -> (restype, argtypes); mirrors include/fwdem.h
SIGNATURES = {
    "fwd_plan_create": (c_int, [POINTER(fwd_plan_desc), POINTER(c_void_p)]),
    "fwd_plan_destroy": (None, [c_void_p]),
    "fwd_set_model": (c_int, [c_void_p, POINTER(c_double)]),
    "fwd_set_model_vti": (c_int, [c_void_p, POINTER(c_double), POINTER(c_double)]),
    "fwd_get_info": (c_int, [c_void_p, POINTER(fwd_info)]),
    "fwd_get_table": (c_int, [c_void_p, c_int, POINTER(c_double), c_size_t]),
    "fwd_workspace_size": (c_int, [c_void_p, c_int, POINTER(c_size_t)]),
    "fwd_volume_size": (c_int, [c_void_p, POINTER(c_size_t)]),
    "fwd_forward": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, c_void_p, c_void_p]),
    "fwd_forward_static": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]),
    "fwd_run_begin": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, c_void_p]),
    "fwd_run_steps": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, c_int, c_void_p]),
    "fwd_run_receivers": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]),
    "fwd_run_flush": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, c_void_p]),
    "fwd_checkpoint_size": (c_int, [c_void_p, c_int, POINTER(c_size_t)]),
    "fwd_checkpoint_save": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, c_void_p,
                                    c_size_t, c_void_p]),
    "fwd_checkpoint_restore": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t,
                                       c_void_p, c_size_t, c_void_p]),
    "fwd_volume_export": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]),
    "fwd_basis_build": (c_int, [c_void_p, c_double, c_double, c_int, c_double,
                                POINTER(c_double), POINTER(c_int)]),
    "fwd_adjoint": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, c_void_p, c_void_p,
                            c_int, c_void_p, c_void_p]),
    "fwd_adjoint_td_size": (c_int, [c_void_p, c_int, POINTER(c_size_t)]),
    "fwd_adjoint_td": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, c_int, c_void_p,
                               c_void_p, c_int, c_void_p]),
    "fwd_set_option": (c_int, [c_void_p, c_int, c_double]),
    "fwd_get_option": (c_int, [c_void_p, c_int, POINTER(c_double)]),
    "fwd_autotune": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, c_int, c_int,
                             POINTER(c_double), c_void_p]),
    "fwd_last_timing": (c_int, [c_void_p, POINTER(c_double), POINTER(c_int)]),
    "fwd_kernel_stats": (c_int, [c_void_p, POINTER(c_double), POINTER(c_int)]),
    "fwd_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libfwdem.so (built by paper_2211_16665_amd.build); raises if it
    is missing -- there is no fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libfwdem.so not built ({path}); run python -m paper_2211_16665_amd.build")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != FWD_OK:
        msg = _lib.fwd_last_error().decode(errors="replace")
        raise FwdError(status, msg)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


def _ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    return None if t is None else c_void_p(t.data_ptr())


def _nbytes(t):
    """Byte count of a torch tensor's storage view (0 for None)."""
    return 0 if t is None else t.numel() * t.element_size()


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return c_void_p(s.cuda_stream)


class Plan:
    """A plan of libfwdem: grid, frequencies, sources and receivers fixed at
    creation; the model set by ``set_model``.  Large device buffers are torch
    tensors owned here or by the caller.  ``rec_comp`` lists the recorded
    components: 0-2 for E_x, E_y, E_z, 3-5 for H_x, H_y, H_z."""

    def __init__(self, x, y, z, freqs, src_pos, src_mom, rec_pos, rec_comp=(0, 1), npml=8,
                 f0=1.0, field_dtype="f32", acc_mode="f64", rho_air_cap=1e4, cfl=0.95,
                 dt=0.0, nt=0, cpml_order=0.0, cpml_R=0.0, cpml_kappa_max=0.0,
                 cpml_alpha_max=0.0, cpml_vref=0.0, fd_order=2, src_kind=0):
        self.lib = load()
        self._keep = [np.ascontiguousarray(a, dtype=np.float64) for a in
                      (x, y, z, freqs, src_pos, src_mom, rec_pos)]
        xx, yy, zz, ff, sp, sm, rp = self._keep
        comp = np.ascontiguousarray(rec_comp, dtype=np.int32)
        self._keep.append(comp)
        d = fwd_plan_desc()
        d.nx, d.ny, d.nz = len(xx) - 1, len(yy) - 1, len(zz) - 1
        d.x, d.y, d.z = _dptr(xx), _dptr(yy), _dptr(zz)
        d.npml = int(npml)
        d.cpml_order, d.cpml_R, d.cpml_kappa_max = cpml_order, cpml_R, cpml_kappa_max
        d.cpml_alpha_max, d.cpml_vref = cpml_alpha_max, cpml_vref
        d.f0 = float(f0)
        d.nfreq, d.freqs = len(ff), _dptr(ff)
        d.nsrc, d.src_pos, d.src_mom = sp.reshape(-1, 3).shape[0], _dptr(sp), _dptr(sm)
        d.nrec, d.rec_pos = rp.reshape(-1, 3).shape[0], _dptr(rp)
        d.ncomp, d.rec_comp = len(comp), comp.ctypes.data_as(POINTER(c_int))
        d.field_dtype = DTYPES[field_dtype]
        d.acc_mode = ACC_MODES[acc_mode]
        d.rho_air_cap, d.cfl, d.dt, d.nt = float(rho_air_cap), float(cfl), float(dt), int(nt)
        d.src_kind = int(src_kind)
        h = c_void_p()
        check(self.lib.fwd_plan_create(byref(d), byref(h)))
        self.handle = h
        self.shape = (d.nz, d.ny, d.nx)
        self.ns, self.nr, self.ncomp, self.nf = d.nsrc, d.nrec, d.ncomp, d.nfreq
        self._ws = None          # the plan's own workspace (both modes; see workspace)
        self._ext_ws = None      # a caller's buffer in its place (use_workspace)
        self.model_serial = 0
        if int(fd_order) != 2:
            self.set_option(FWD_OPT_FD_ORDER, int(fd_order))

    @classmethod
    def from_workload(cls, w, field_dtype=None, acc_mode=None, **kw):
        args = dict(npml=w.npml, f0=w.f0, rho_air_cap=w.rho_air_cap, cfl=w.cfl, dt=w.dt,
                    nt=w.nt, field_dtype=field_dtype or w.field_dtype,
                    acc_mode=acc_mode or w.acc_mode, fd_order=getattr(w, "fd_order", 2),
                    src_kind=getattr(w, "src_kind", 0))
        for k in ("cpml_order", "cpml_R", "cpml_kappa_max", "cpml_alpha_max", "cpml_vref"):
            if hasattr(w, k):
                args[k] = getattr(w, k)
        args.update(kw)
        return cls(w.x, w.y, w.z, w.freqs, w.src_pos, w.src_mom, w.rec_pos, w.rec_comp, **args)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                import torch
                if torch.cuda.is_available():
                    torch.cuda.synchronize()
            except Exception:
                pass
            self.lib.fwd_plan_destroy(h)
            self.handle = None

    # ---- host-side calls --------------------------------------------------
    def set_model(self, rho, rho_v=None):
        """Cell resistivity [nz][ny][nx]; with ``rho_v`` a VTI model (rho is
        then the horizontal resistivity).  ``model_serial`` counts the
        calls (and order changes, which drop the model)."""
        self.model_serial += 1
        r = np.ascontiguousarray(np.asarray(rho, dtype=np.float64))
        if r.shape != self.shape:
            raise ValueError(f"rho must have shape {self.shape}")
        if rho_v is None:
            check(self.lib.fwd_set_model(self.handle, _dptr(r)))
            return
        rv = np.ascontiguousarray(np.asarray(rho_v, dtype=np.float64))
        if rv.shape != self.shape:
            raise ValueError(f"rho_v must have shape {self.shape}")
        check(self.lib.fwd_set_model_vti(self.handle, _dptr(r), _dptr(rv)))

    @property
    def grad_shape(self):
        """Shape of a gradient: (nz, ny, nx), or (2, nz, ny, nx) for the split
        VTI gradient (FWD_OPT_VTI_GRADIENT = 1)."""
        return ((2,) + self.shape) if self.get_option(FWD_OPT_VTI_GRADIENT) else self.shape

    @property
    def info(self) -> fwd_info:
        i = fwd_info()
        check(self.lib.fwd_get_info(self.handle, byref(i)))
        return i

    def table(self, which: int, n: int) -> np.ndarray:
        out = np.zeros(n)
        check(self.lib.fwd_get_table(self.handle, which, _dptr(out), n))
        return out

    def basis_build(self, gamma_rel=1e-12, gamma_abs=0.0, max_iter=2000, tol=1e-13):
        fit, it = c_double(), c_int()
        check(self.lib.fwd_basis_build(self.handle, gamma_rel, gamma_abs, max_iter, tol,
                                       byref(fit), byref(it)))
        return fit.value, it.value

    def set_option(self, key: int, value: float):
        if key == FWD_OPT_FD_ORDER:
            self.model_serial += 1
        check(self.lib.fwd_set_option(self.handle, key, float(value)))

    def get_option(self, key: int) -> float:
        v = c_double()
        check(self.lib.fwd_get_option(self.handle, key, byref(v)))
        return v.value

    # ---- device buffers ----------------------------------------------------
    def workspace_size(self, mode=FWD_MODE_FORWARD) -> int:
        n = c_size_t()
        check(self.lib.fwd_workspace_size(self.handle, mode, byref(n)))
        return n.value

    def volume_size(self) -> int:
        n = c_size_t()
        check(self.lib.fwd_volume_size(self.handle, byref(n)))
        return n.value

    def use_workspace(self, buf):
        """Run on the caller's device buffer ``buf`` (uint8 tensor) instead of
        a workspace owned by the plan -- e.g. one buffer for several plans run
        one after the other on one stream; None returns to the plan's own."""
        self._ext_ws = buf
        self._ws = None

    def workspace(self, mode=FWD_MODE_FORWARD):
        """Device workspace of a ``mode`` run.  One buffer serves both modes
        (the runs of a plan are enqueued on one stream and never overlap; each
        run starts by zeroing the state it uses), grown to the largest size
        asked for."""
        import torch
        need = self.workspace_size(mode)
        if self._ext_ws is not None:
            if self._ext_ws.numel() < need:
                raise ValueError(f"external workspace holds {self._ext_ws.numel()} bytes, "
                                 f"the run needs {need}")
            return self._ext_ws
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        return self._ws

    def volume_buffer(self):
        import torch
        return torch.empty(self.volume_size(), dtype=torch.uint8, device="cuda")

    def rec_buffer(self):
        import torch
        return torch.empty((self.ns, self.nr, self.ncomp, self.nf), dtype=torch.complex128,
                           device="cuda")

    # ---- device calls ------------------------------------------------------
    def forward(self, vol=None, want_volume=False, stream=None):
        """E at the receivers, complex128 [ns][nr][ncomp][nf]; with
        ``want_volume`` also the raw volume transform (uint8 tensor)."""
        ws = self.workspace(FWD_MODE_FORWARD)
        if want_volume and vol is None:
            vol = self.volume_buffer()
        E = self.rec_buffer()
        check(self.lib.fwd_forward(self.handle, _ptr(ws), ws.numel(), _ptr(vol),
                                   0 if vol is None else vol.numel(), _ptr(E), _stream(stream)))
        return (E, vol) if want_volume else E

    def forward_static(self, vol=None, out=None, stream=None):
        """fwd_forward_static: the forward run with the workspace in the
        library's static device array (no device allocation inside the
        call; ``out``, a complex128 [ns][nr][ncomp][nf] tensor, avoids the
        binding's own).  The plan's tables must be resident: call
        ``forward`` once first."""
        E = self.rec_buffer() if out is None else out
        check(self.lib.fwd_forward_static(self.handle, _ptr(vol), 0 if vol is None else vol.numel(),
                                          _ptr(E), _stream(stream)))
        return E

    def run_begin(self, vol=None, stream=None):
        ws = self.workspace(FWD_MODE_FORWARD)
        check(self.lib.fwd_run_begin(self.handle, _ptr(ws), ws.numel(), _ptr(vol),
                                     0 if vol is None else vol.numel(), _stream(stream)))

    def run_steps(self, nsteps, vol=None, stream=None):
        ws = self.workspace(FWD_MODE_FORWARD)
        check(self.lib.fwd_run_steps(self.handle, _ptr(ws), ws.numel(), _ptr(vol), _nbytes(vol),
                                     int(nsteps), _stream(stream)))

    def run_receivers(self, stream=None):
        ws = self.workspace(FWD_MODE_FORWARD)
        E = self.rec_buffer()
        check(self.lib.fwd_run_receivers(self.handle, _ptr(ws), ws.numel(), _ptr(E),
                                         _stream(stream)))
        return E

    def run_flush(self, vol, stream=None):
        ws = self.workspace(FWD_MODE_FORWARD)
        check(self.lib.fwd_run_flush(self.handle, _ptr(ws), ws.numel(), _ptr(vol), _nbytes(vol),
                                     _stream(stream)))

    def checkpoint_size(self, with_volume=False) -> int:
        n = c_size_t()
        check(self.lib.fwd_checkpoint_size(self.handle, int(with_volume), byref(n)))
        return n.value

    def checkpoint_save(self, snap, vol=None, stream=None):
        ws = self.workspace(FWD_MODE_FORWARD)
        check(self.lib.fwd_checkpoint_save(self.handle, _ptr(ws), ws.numel(), _ptr(vol),
                                           _nbytes(vol), _ptr(snap), _nbytes(snap),
                                           _stream(stream)))

    def checkpoint_restore(self, snap, vol=None, stream=None):
        ws = self.workspace(FWD_MODE_FORWARD)
        check(self.lib.fwd_checkpoint_restore(self.handle, _ptr(ws), ws.numel(), _ptr(vol),
                                              _nbytes(vol), _ptr(snap), _nbytes(snap),
                                              _stream(stream)))

    def volume_export(self, vol, stream=None):
        import torch
        nz, ny, nx = self.shape
        out = torch.empty((self.ns, self.nf, 3, nz + 1, ny + 1, nx + 1), dtype=torch.complex128,
                          device="cuda")
        check(self.lib.fwd_volume_export(self.handle, _ptr(vol), _nbytes(vol), _ptr(out),
                                         _stream(stream)))
        return out

    def adjoint(self, vol, resid, grad=None, accumulate=False, want_adjoint_rec=False,
                stream=None):
        """Gradient d phi / d ln rho [nz][ny][nx] (float64) for the weighted
        residual ``resid`` = W^2 (d - E), complex128 [ns][nr][ncomp][nf]."""
        import torch
        ws = self.workspace(FWD_MODE_ADJOINT)
        resid = resid.to(device="cuda", dtype=torch.complex128).contiguous()
        if grad is None:
            grad = torch.zeros(self.grad_shape, dtype=torch.float64, device="cuda")
        elif tuple(grad.shape) != tuple(self.grad_shape) or grad.dtype != torch.float64:
            raise ValueError(f"grad must be float64 of shape {self.grad_shape}")
        Ea = self.rec_buffer() if want_adjoint_rec else None
        check(self.lib.fwd_adjoint(self.handle, _ptr(ws), ws.numel(), _ptr(vol), _nbytes(vol),
                                   _ptr(resid), _ptr(grad), int(accumulate), _ptr(Ea),
                                   _stream(stream)))
        return (grad, Ea) if want_adjoint_rec else grad

    def adjoint_td_size(self, segment=200):
        n = c_size_t()
        check(self.lib.fwd_adjoint_td_size(self.handle, int(segment), ctypes.byref(n)))
        return n.value

    def adjoint_td(self, resid, grad=None, accumulate=False, segment=200, scratch=None,
                   stream=None):
        """Gradient d phi / d ln rho [nz][ny][nx] (float64) by the time-domain
        adjoint (checkpoints every ``segment`` steps) for the weighted
        residual ``resid`` = W^2 (d - E), complex128 [ns][nr][ncomp][nf]."""
        import torch
        ws = self.workspace(FWD_MODE_FORWARD)
        need = self.adjoint_td_size(segment)
        if scratch is None or scratch.numel() < need:
            scratch = torch.empty(need, dtype=torch.uint8, device="cuda")
        resid = resid.to(device="cuda", dtype=torch.complex128).contiguous()
        if grad is None:
            grad = torch.zeros(self.grad_shape, dtype=torch.float64, device="cuda")
        elif tuple(grad.shape) != tuple(self.grad_shape) or grad.dtype != torch.float64:
            raise ValueError(f"grad must be float64 of shape {self.grad_shape}")
        check(self.lib.fwd_adjoint_td(self.handle, _ptr(ws), ws.numel(), _ptr(scratch),
                                      scratch.numel(), int(segment), _ptr(resid), _ptr(grad),
                                      int(accumulate), _stream(stream)))
        return grad

    def autotune(self, mode=FWD_MODE_FORWARD, vol=None, steps=20, stream=None):
        ws = self.workspace(mode)
        ms = c_double()
        check(self.lib.fwd_autotune(self.handle, _ptr(ws), ws.numel(), _ptr(vol),
                                    0 if vol is None else vol.numel(), mode, int(steps),
                                    byref(ms), _stream(stream)))
        return ms.value

    def last_timing(self):
        ms, n = c_double(), c_int()
        check(self.lib.fwd_last_timing(self.handle, byref(ms), byref(n)))
        return ms.value, n.value

    def kernel_stats(self):
        """([H update, E update, block transform] average ms per launch, sampled
        steps) of the last forward / adjoint (FWD_OPT_SAMPLE_EVERY > 0)."""
        arr = (c_double * 3)()
        n = c_int()
        check(self.lib.fwd_kernel_stats(self.handle, arr, byref(n)))
        return list(arr), n.value
