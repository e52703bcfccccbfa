"""Python face of the C ABI: a ``Solver`` owning one library context.

Only marshalling happens here (shape, dtype, device and contiguity checks,
pointer and stream hand-over); every step of the computation runs in the HIP
kernels of ``libins.so``. torch supplies device memory and the stream.
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import _lib as L

_DTYPES = {"fp64": (L.INS_FP64, torch.float64), "fp32": (L.INS_FP32, torch.float32),
           "fp32_all": (L.INS_FP32_ALL, torch.float32)}
_BCS = {"periodic": L.INS_BC_PERIODIC, "walls": L.INS_BC_WALLS_Y}
_PRESSURE = {"auto": L.INS_PRESSURE_AUTO, "fft": L.INS_PRESSURE_FFT, "cg": L.INS_PRESSURE_CG}


class Solver:
    """Staggered-grid incompressible Navier-Stokes operators on one GPU.

    Args:
        n: cells per direction, (n_x, n_y) or (n_x, n_y, n_z).
        nu: kinematic viscosity.
        precision: "fp64" (everything float64), "fp32" (float32 velocity
            fields, stencils and RK stages; float64 divergence, Poisson solve
            and projection) or "fp32_all" (for comparison: everything float32,
            pressure-point fields and the FFT solve included; periodic grid,
            forward operators and steps only).
        batch: number of independent fields per call.
        lo, hi: box corners (default [0, 2 pi] per direction).
        bc: "periodic" (every direction; FFT pressure solve) or "walls"
            (channel: no-slip walls at y = lo[1] and hi[1], x and z periodic).
            In the channel the stored u^y face of the last cell row is the
            upper wall: it reads as 0 and every output writes 0 there.
        pressure: the pressure solver. "auto" (default): FFT where it applies,
            else CG; "fft": spectral (channel: FFTs along x and z and a direct
            tridiagonal solve along y per mode); "cg": matrix-free conjugate
            gradients (channel only, see cg_set).
    """

    def __init__(self, n, nu=0.0, precision="fp64", batch=1, lo=None, hi=None, device=None, bc="periodic",
                 pressure="auto"):
        if precision not in _DTYPES:
            raise ValueError(f"precision must be one of {list(_DTYPES)}")
        if bc not in _BCS:
            raise ValueError(f"bc must be one of {list(_BCS)}")
        self.bc = bc
        self.n = tuple(int(v) for v in n)
        self.dim = len(self.n)
        if self.dim not in (2, 3):
            raise ValueError("n must have 2 or 3 entries")
        self.nu = float(nu)
        self.batch = int(batch)
        self.precision = precision
        self._code, self.dtype = _DTYPES[precision]
        # pressure-point fields: float64, float32 in the all-float32 comparison mode
        self.pdtype = torch.float32 if precision == "fp32_all" else torch.float64
        self.lo = tuple(float(v) for v in (lo if lo is not None else [0.0] * self.dim))
        self.hi = tuple(float(v) for v in (hi if hi is not None else [2 * math.pi] * self.dim))
        self.h = tuple((self.hi[a] - self.lo[a]) / self.n[a] for a in range(self.dim))
        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a HIP device (torch.cuda.is_available() is False)")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else torch.device(device).index or 0)
        g = L.Grid()
        g.dim = self.dim
        for a in range(3):
            g.n[a] = self.n[a] if a < self.dim else 1
            g.lo[a] = self.lo[a] if a < self.dim else 0.0
            g.hi[a] = self.hi[a] if a < self.dim else 1.0
        g.batch = self.batch
        self._ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            L.call("ins_create", C.byref(g), _BCS[bc], self.nu, self._code, C.byref(self._ctx))
        if pressure != "auto":
            self.set_pressure(pressure)
        spatial = tuple(reversed(self.n))
        self.vel_shape = (self.batch, self.dim) + spatial
        self.scal_shape = (self.batch,) + spatial

    # ------------------------------------------------------------------ utils
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            L.call("ins_destroy", self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        L.call("ins_set_stream", self._ctx, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def _check(self, t, kind, name):
        shape = self.vel_shape if kind == "vel" else self.scal_shape
        dtype = self.dtype if kind == "vel" else self.pdtype
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}, got {t.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != shape and not (self.batch == 1 and tuple(t.shape) == shape[1:]):
            raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return C.c_void_p(t.data_ptr())

    def _unbatched(self, t):
        return self.batch == 1 and t is not None and t.dim() in (len(self.vel_shape) - 1, len(self.scal_shape) - 1) \
            and tuple(t.shape) in (self.vel_shape[1:], self.scal_shape[1:])

    def _out(self, out, like, kind):
        if out is None:
            shape = self.vel_shape if kind == "vel" else self.scal_shape
            if self._unbatched(like):
                shape = shape[1:]
            dtype = self.dtype if kind == "vel" else self.pdtype
            return torch.empty(shape, dtype=dtype, device=self.device)
        return out

    def new_velocity(self, fill=None):
        t = torch.empty(self.vel_shape, dtype=self.dtype, device=self.device)
        return t.zero_() if fill is None else t.fill_(fill)

    def new_scalar(self):
        return torch.zeros(self.scal_shape, dtype=self.pdtype, device=self.device)

    def set_pressure(self, solver):
        """Pressure solver for later calls: "auto", "fft" or "cg"."""
        if solver not in _PRESSURE:
            raise ValueError(f"pressure must be one of {list(_PRESSURE)}")
        L.call("ins_set_pressure_solver", self._ctx, _PRESSURE[solver])

    @property
    def pressure(self):
        """The pressure solver in use, "fft" or "cg"."""
        v = C.c_int()
        L.call("ins_get_pressure_solver", self._ctx, C.byref(v))
        return "cg" if v.value == L.INS_PRESSURE_CG else "fft"

    def set_body_force(self, force):
        """Constant body force (dim values) added to F on the channel, e.g. (1, 0, 0)."""
        if len(force) != self.dim:
            raise ValueError(f"force must have {self.dim} components")
        f = (C.c_double * self.dim)(*[float(v) for v in force])
        L.call("ins_set_body_force", self._ctx, f)
        self.body_force = tuple(float(v) for v in force)

    def cg_set(self, rtol=1e-10, maxiter=20000, check_every=16):
        """Stopping rule of the channel's conjugate-gradient pressure solves."""
        L.call("ins_cg_set", self._ctx, float(rtol), int(maxiter), int(check_every))

    def set_y_faces(self, faces):
        """Stretch the channel's y grid: the n_y + 1 face coordinates (host values, increasing)."""
        import numpy as _np

        f = _np.ascontiguousarray(_np.asarray(faces, dtype=_np.float64))
        if f.shape != (self.n[1] + 1,):
            raise ValueError(f"faces must hold n_y + 1 = {self.n[1] + 1} coordinates")
        self._sync_stream()
        L.call("ins_set_y_faces", self._ctx, f.ctypes.data_as(C.POINTER(C.c_double)))
        self.y_faces = f.copy()

    def set_faces(self, axis, faces):
        """Stretch direction ``axis`` (0 = x, 1 = y, 2 = z): its n + 1 face coordinates
        (host values, increasing). A periodic direction wraps with the period
        faces[-1] - faces[0]. Stretching a periodic direction switches the solver to
        the stretched-grid kernels and the CG pressure solve for good."""
        import numpy as _np

        axis = int(axis)
        if not 0 <= axis < self.dim:
            raise ValueError("axis must be 0 .. dim - 1")
        f = _np.ascontiguousarray(_np.asarray(faces, dtype=_np.float64))
        if f.shape != (self.n[axis] + 1,):
            raise ValueError(f"faces must hold n + 1 = {self.n[axis] + 1} coordinates")
        self._sync_stream()
        L.call("ins_set_faces", self._ctx, axis, f.ctypes.data_as(C.POINTER(C.c_double)))
        if axis == 1:
            self.y_faces = f.copy()

    def cg_info(self):
        """(iterations, relative residual) of the last pressure solve (maxima over the batch)."""
        self._sync_stream()
        it, rel = C.c_int(), C.c_double()
        L.call("ins_cg_info", self._ctx, C.byref(it), C.byref(rel))
        return int(it.value), float(rel.value)

    def workspace_bytes(self):
        v = C.c_size_t()
        L.call("ins_workspace_bytes", self._ctx, C.byref(v))
        return int(v.value)

    # -------------------------------------------------------------- forward
    def rhs(self, u, out=None):
        out = self._out(out, u, "vel")
        self._sync_stream()
        L.call("ins_rhs", self._ctx, self._check(u, "vel", "u"), self._check(out, "vel", "out"))
        return out

    def divergence(self, u, out=None):
        out = self._out(out, u, "scal")
        self._sync_stream()
        L.call("ins_divergence", self._ctx, self._check(u, "vel", "u"), self._check(out, "scal", "out"))
        return out

    def gradient(self, p, out=None):
        out = self._out(out, p, "vel")
        self._sync_stream()
        L.call("ins_gradient", self._ctx, self._check(p, "scal", "p"), self._check(out, "vel", "out"))
        return out

    def poisson_solve(self, r, out=None):
        out = self._out(out, r, "scal")
        self._sync_stream()
        L.call("ins_poisson_solve", self._ctx, self._check(r, "scal", "r"), self._check(out, "scal", "out"))
        return out

    def project(self, u, out=None, p_out=None):
        out = self._out(out, u, "vel")
        self._sync_stream()
        pp = self._check(p_out, "scal", "p_out") if p_out is not None else None
        L.call("ins_project", self._ctx, self._check(u, "vel", "u"), self._check(out, "vel", "out"), pp)
        return out

    _SCHEMES = {"rk4": ("ins_step_rk4", "ins_step_rk4_vjp"), "wray3": ("ins_step_wray3", "ins_step_wray3_vjp")}

    def _scheme(self, scheme):
        if scheme not in self._SCHEMES:
            raise ValueError(f"scheme must be one of {sorted(self._SCHEMES)}")
        return self._SCHEMES[scheme]

    _SCHEME_IDS = {"rk4": 0, "wray3": 1}

    def stage_buffers(self, scheme="rk4"):
        """(stages, pstages) buffers for step(..., keep=) / step_vjp(..., kept=)."""
        k = L.load().ins_scheme_stage_count(self._SCHEME_IDS[scheme])
        stages = torch.empty((k,) + self.vel_shape, dtype=self.dtype, device=self.device)
        pstages = torch.empty((k,) + self.scal_shape, dtype=torch.float64, device=self.device)
        return stages, pstages

    def _kept(self, kept, scheme):
        stages, pstages = kept
        k = L.load().ins_scheme_stage_count(self._SCHEME_IDS[scheme])
        if (not isinstance(stages, torch.Tensor) or tuple(stages.shape) != (k,) + self.vel_shape
                or stages.dtype != self.dtype or stages.device != self.device or not stages.is_contiguous()):
            raise ValueError("stages must come from stage_buffers(scheme)")
        if (not isinstance(pstages, torch.Tensor) or tuple(pstages.shape) != (k,) + self.scal_shape
                or pstages.dtype != torch.float64 or pstages.device != self.device or not pstages.is_contiguous()):
            raise ValueError("pstages must come from stage_buffers(scheme)")
        return stages.data_ptr(), pstages.data_ptr()

    def step(self, u0, dt, out=None, scheme="rk4", keep=None):
        """One time step (classical RK4, or Wray's low-storage RK3 with scheme="wray3");
        out may be u0 (in place). keep=(stages, pstages) from stage_buffers() keeps the
        stage inputs there for step_vjp(..., kept=)."""
        fn = self._scheme(scheme)[0]
        out = self._out(out, u0, "vel")
        self._sync_stream()
        if keep is None:
            L.call(fn, self._ctx, self._check(u0, "vel", "u0"), self._check(out, "vel", "out"), float(dt))
        else:
            sp, pp = self._kept(keep, scheme)
            L.call("ins_step_save", self._ctx, self._SCHEME_IDS[scheme], self._check(u0, "vel", "u0"),
                   self._check(out, "vel", "out"), float(dt), sp, pp)
        return out

    # ------------------------------------------------------------- pullbacks
    def rhs_vjp(self, u, fbar, out=None):
        out = self._out(out, u, "vel")
        self._sync_stream()
        L.call("ins_rhs_vjp", self._ctx, self._check(u, "vel", "u"), self._check(fbar, "vel", "fbar"),
               self._check(out, "vel", "out"))
        return out

    def divergence_vjp(self, rbar, out=None):
        out = self._out(out, rbar, "vel")
        self._sync_stream()
        L.call("ins_divergence_vjp", self._ctx, self._check(rbar, "scal", "rbar"), self._check(out, "vel", "out"))
        return out

    def gradient_vjp(self, gbar, out=None):
        out = self._out(out, gbar, "scal")
        self._sync_stream()
        L.call("ins_gradient_vjp", self._ctx, self._check(gbar, "vel", "gbar"), self._check(out, "scal", "out"))
        return out

    def poisson_solve_vjp(self, pbar, out=None):
        out = self._out(out, pbar, "scal")
        self._sync_stream()
        L.call("ins_poisson_solve_vjp", self._ctx, self._check(pbar, "scal", "pbar"), self._check(out, "scal", "out"))
        return out

    def project_vjp(self, ubar_out, out=None):
        out = self._out(out, ubar_out, "vel")
        self._sync_stream()
        L.call("ins_project_vjp", self._ctx, self._check(ubar_out, "vel", "ubar_out"), self._check(out, "vel", "out"))
        return out

    def step_vjp(self, u0, u1bar, dt, out=None, scheme="rk4", kept=None):
        """(d u1 / d u0)^T u1bar; kept=(stages, pstages) filled by step(u0, dt, keep=) skips
        the recomputation of the stage inputs."""
        fn = self._scheme(scheme)[1]
        out = self._out(out, u0, "vel")
        self._sync_stream()
        if kept is not None:
            sp, pp = self._kept(kept, scheme)
            L.call("ins_step_vjp_saved", self._ctx, self._SCHEME_IDS[scheme], self._check(u0, "vel", "u0"), sp, pp,
                   self._check(u1bar, "vel", "u1bar"), self._check(out, "vel", "out"), float(dt))
            return out
        L.call(fn, self._ctx, self._check(u0, "vel", "u0"), self._check(u1bar, "vel", "u1bar"),
               self._check(out, "vel", "out"), float(dt))
        return out

    # ------------------------------------------------------- learned closure
    N_CLOSURE_PARAMS = 32899

    def _params(self, t, name):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or t.device != self.device \
                or t.numel() != self.N_CLOSURE_PARAMS or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 tensor of {self.N_CLOSURE_PARAMS} values on {self.device}")
        return C.c_void_p(t.data_ptr())

    def set_closure(self, params):
        """Attach the CNN closure with float32 parameters (None detaches it)."""
        self._sync_stream()
        L.call("ins_closure_set", self._ctx, None if params is None else self._params(params, "params"))

    def closure_grad(self, out=None):
        """Parameter gradient accumulated by the *_vjp calls since the last read (resets it)."""
        out = torch.empty(self.N_CLOSURE_PARAMS, dtype=torch.float32, device=self.device) if out is None else out
        self._sync_stream()
        L.call("ins_closure_grad", self._ctx, self._params(out, "out"))
        return out

    def cnn_forward(self, u, out=None):
        out = self._out(out, u, "vel")
        self._sync_stream()
        L.call("ins_cnn_forward", self._ctx, self._check(u, "vel", "u"), self._check(out, "vel", "out"))
        return out

    def cnn_backward(self, u, mbar):
        """(ubar, params_bar) of the closure alone."""
        ubar = self._out(None, u, "vel")
        pbar = torch.empty(self.N_CLOSURE_PARAMS, dtype=torch.float32, device=self.device)
        self._sync_stream()
        L.call("ins_cnn_backward", self._ctx, self._check(u, "vel", "u"), self._check(mbar, "vel", "mbar"),
               self._check(ubar, "vel", "ubar"), self._params(pbar, "params_bar"))
        return ubar, pbar

    _CNN_SAVED = {0: (8, torch.int16), 1: (32, torch.float32), 2: (32, torch.int16), 3: (32, torch.float32),
                  4: (32, torch.int16), 5: (8, torch.int16), 6: (32, torch.int16), 7: (32, torch.int16)}

    def cnn_saved(self, which):
        """Copy of one of the closure's internal tensors after cnn_backward
        (see ins_cnn_saved): channels-last [cells][C]; bfloat16 tensors are
        returned as torch.bfloat16, which = 8 gives m in the field layout."""
        if which == 8:
            out = self._out(None, None, "vel")
        else:
            ch, dt = self._CNN_SAVED[which]
            ncell = self.batch * math.prod(self.n)
            out = torch.empty((ncell, ch), dtype=dt, device=self.device)
        self._sync_stream()
        L.call("ins_cnn_saved", self._ctx, int(which), C.c_void_p(out.data_ptr()))
        return out.view(torch.bfloat16) if out.dtype == torch.int16 else out

    # ------------------------------------------------ Smagorinsky closure
    def set_eddy(self, cs=0.17, delta=None):
        """Attach the Smagorinsky eddy-viscosity closure (cs = 0 detaches it);
        delta = None takes the geometric mean of the spacings as filter width."""
        self._sync_stream()
        L.call("ins_eddy_set", self._ctx, float(cs), 0.0 if delta is None else float(delta))

    def eddy_forward(self, u, out=None):
        out = self._out(out, u, "vel")
        self._sync_stream()
        L.call("ins_eddy_forward", self._ctx, self._check(u, "vel", "u"), self._check(out, "vel", "out"))
        return out

    def eddy_backward(self, u, mbar, out=None):
        out = self._out(out, u, "vel")
        self._sync_stream()
        L.call("ins_eddy_backward", self._ctx, self._check(u, "vel", "u"), self._check(mbar, "vel", "mbar"),
               self._check(out, "vel", "out"))
        return out

    # ------------------------------------------------------- LES data helpers
    def face_filter(self, u, factor=4, out=None):
        """Coarse staggered field: mean of the fine faces on each coarse face."""
        if out is None:
            cn = tuple(v // factor for v in reversed(self.n))
            shape = (self.dim,) + cn if self._unbatched(u) else (self.batch, self.dim) + cn
            out = torch.empty(shape, dtype=self.dtype, device=self.device)
        if out.dtype != self.dtype or not out.is_contiguous() or out.numel() * factor ** self.dim != self.batch * self.dim * math.prod(self.n):
            raise ValueError("out must be a contiguous coarse field of the solver dtype")
        self._sync_stream()
        L.call("ins_face_filter", self._ctx, self._check(u, "vel", "u"), int(factor), C.c_void_p(out.data_ptr()))
        return out

    def spectrum_bins(self):
        return int(math.floor(math.sqrt(self.dim) * max(self.n) / 2 + 0.5)) + 1

    def energy_spectrum(self, u, nbins=None):
        """E(k), k = 0..nbins-1 (float64, shape (batch, nbins), or (nbins,) for an unbatched input)."""
        nbins = self.spectrum_bins() if nbins is None else int(nbins)
        e = torch.empty((self.batch, nbins), dtype=torch.float64, device=self.device)
        self._sync_stream()
        L.call("ins_energy_spectrum", self._ctx, self._check(u, "vel", "u"), C.c_void_p(e.data_ptr()), nbins)
        return e[0] if self._unbatched(u) else e

    # ------------------------------------------------------------ utilities
    def stats(self, u):
        """(kinetic energy, max|u|, max|Du|, all finite) of a velocity field."""
        out = (C.c_double * 4)()
        self._sync_stream()
        L.call("ins_stats", self._ctx, self._check(u, "vel", "u"), out)
        return float(out[0]), float(out[1]), float(out[2]), bool(out[3] != 0.0)

    def stats_noalloc(self, u, out):
        """The statistics of ``stats`` written to ``out`` (a float64 device tensor of
        4 values: kinetic energy, max|u|, max|Du|, 1.0 if all finite) without
        allocating or synchronising; calls on one device must not overlap."""
        if not isinstance(out, torch.Tensor) or out.dtype != torch.float64 or out.device != self.device \
                or out.numel() != 4 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of 4 values on the solver's device")
        self._sync_stream()
        L.call("ins_stats_noalloc", self._ctx, self._check(u, "vel", "u"), C.c_void_p(out.data_ptr()))
        return out

    def stream_copy(self, src, dst):
        if src.numel() * src.element_size() != dst.numel() * dst.element_size():
            raise ValueError("size mismatch")
        self._sync_stream()
        L.call("ins_stream_copy", self._ctx, C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
               src.numel() * src.element_size())

    def profile(self, enable=True):
        L.call("ins_profile_enable", self._ctx, 1 if enable else 0)

    def profile_reset(self):
        L.call("ins_profile_reset", self._ctx)

    def profile_read(self):
        """{kernel name: (launches, total ms)} since the last reset (synchronises)."""
        cnt = C.c_int()
        L.call("ins_profile_count", self._ctx, C.byref(cnt))
        res = {}
        buf = C.create_string_buffer(128)
        for i in range(cnt.value):
            nl, ms = C.c_int64(), C.c_double()
            L.call("ins_profile_read", self._ctx, i, buf, 128, C.byref(nl), C.byref(ms))
            res[buf.value.decode()] = (int(nl.value), float(ms.value))
        return res
