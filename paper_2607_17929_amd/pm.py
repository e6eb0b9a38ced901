"""Python binding of the PM library: same call names as the C ABI, argument marshalling only.

PyTorch provides the device workspace and the stream; every step of the
particle-mesh path runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L

_PHYS = {"newtonian": L.PM_NEWTONIAN, "scalar": L.PM_SCALAR, "full": L.PM_FULL}
_PREC = {"fp32": L.PM_FP32, "fp64": L.PM_FP64}


def make_config(n_mesh: int, n_particles: int, box_mpch: float, physics: str = "full", precision: str = "fp32",
                timings: bool = False, closure: bool = False, b_route: str = "elliptic", n_particles_2: int = 0,
                mass_fraction_2: float = 0.0, deterministic: bool = False) -> L.PMConfig:
    if b_route not in ("elliptic", "parabolic"):
        raise ValueError("b_route must be 'elliptic' or 'parabolic'")
    flags = ((L.PM_FLAG_TIMINGS if timings else 0) | (L.PM_FLAG_CLOSURE if closure else 0)
             | (L.PM_FLAG_B_PARABOLIC if b_route == "parabolic" else 0)
             | (L.PM_FLAG_DETERMINISTIC if deterministic else 0))
    return L.PMConfig(n_mesh=n_mesh, precision=_PREC[precision], n_particles=n_particles, box_mpch=box_mpch,
                      physics=_PHYS[physics], flags=flags, n_particles_2=n_particles_2,
                      mass_fraction_2=mass_fraction_2)


def query_workspace(cfg: L.PMConfig) -> int:
    lib = L.load()
    b = C.c_size_t(0)
    L.check(lib.pm_query_workspace(C.byref(cfg), C.byref(b)), what="pm_query_workspace")
    return int(b.value)


def background(box_mpch: float, tau: float):
    """(a, H_conf) of the library's Einstein-de Sitter background at conformal time tau."""
    lib = L.load()
    cfg = make_config(16, 1, box_mpch)
    a, h = C.c_double(), C.c_double()
    L.check(lib.pm_background(C.byref(cfg), tau, C.byref(a), C.byref(h)), what="pm_background")
    return a.value, h.value


def tau_of_a(box_mpch: float, a: float) -> float:
    lib = L.load()
    cfg = make_config(16, 1, box_mpch)
    t = C.c_double()
    L.check(lib.pm_tau_of_a(C.byref(cfg), a, C.byref(t)), what="pm_tau_of_a")
    return t.value


def copy_probe(nbytes: int = 2 ** 31, reps: int = 5, device: str | torch.device = "cuda:0") -> float:
    """Sustainable device copy rate (read + write bytes per second) from the library's copy kernel
    (pm_copy_probe) on two buffers of nbytes."""
    lib = L.load()
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=device)
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream(torch.device(device))
    ms = C.c_double()
    L.check(lib.pm_copy_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes, reps,
                              C.c_void_p(st.cuda_stream), C.byref(ms)), what="pm_copy_probe")
    if not torch.equal(src[:1024], dst[:1024]) or not torch.equal(src[-1024:], dst[-1024:]):
        raise RuntimeError("pm_copy_probe did not copy")
    return 2.0 * nbytes / (ms.value * 1e-3)


def fft_noalloc(x: torch.Tensor, n: int, direction: int, precision: str = "fp32") -> torch.Tensor:
    """pm_fft_noalloc: the context-free FFT of pm_debug_fft (scratch in the library's fixed device array);
    the output tensor is allocated here, by the caller's side."""
    lib = L.load()
    rdt = torch.float64 if precision == "fp64" else torch.float32
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    if direction == 1:
        x = x.to(dtype=rdt).contiguous()
        out = torch.empty((n, n, n // 2 + 1), dtype=cdt, device=x.device)
    else:
        x = x.to(dtype=cdt).contiguous()
        out = torch.empty((n, n, n), dtype=rdt, device=x.device)
    st = torch.cuda.current_stream(x.device)
    L.check(lib.pm_fft_noalloc(C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), n, _PREC[precision], direction,
                               C.c_void_p(st.cuda_stream)), what="pm_fft_noalloc")
    return out


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


class PMContext:
    """One particle-mesh simulation on one GPU (wraps pm_ctx)."""

    def __init__(self, n_mesh: int, n_particles: int, box_mpch: float, physics: str = "full",
                 precision: str = "fp32", timings: bool = False, device: str | torch.device = "cuda:0",
                 stream: torch.cuda.Stream | None = None, closure: bool = False, b_route: str = "elliptic",
                 n_particles_2: int = 0, mass_fraction_2: float = 0.0, deterministic: bool = False):
        self.lib = L.load()
        self.cfg = make_config(n_mesh, n_particles, box_mpch, physics, precision, timings, closure, b_route,
                               n_particles_2, mass_fraction_2, deterministic)
        self.n = n_mesh
        self.np = n_particles
        self.np2 = n_particles_2
        self.physics = physics
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.np_dtype = np.float64 if precision == "fp64" else np.float32
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ws_bytes = query_workspace(self.cfg)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.ctx = C.c_void_p()
        L.check(self.lib.pm_create(C.byref(self.cfg), C.c_void_p(_ptr(self.workspace)), self.ws_bytes,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(self.ctx)), what="pm_create")

    def close(self):
        if self.ctx:
            self.lib.pm_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, status, what):
        L.check(status, self.ctx, what)

    # -- the five calls of the boundary -----------------------------------
    def init_particles(self, pos, u, tau0: float, ids=None):
        """pos [n][3] float64, u [n][3] context precision; numpy (host) or CUDA tensors (device)."""
        if isinstance(pos, torch.Tensor):
            if not (pos.is_cuda and u.is_cuda):
                raise ValueError("pos and u must both be device tensors or both numpy arrays")
            pos = pos.to(torch.float64).contiguous()
            u = u.to(self.dtype).contiguous()
            idp = ids.to(torch.int32).contiguous() if ids is not None else None
            self._keep = (pos, u, idp)
            self._chk(self.lib.pm_init_particles(self.ctx, C.c_void_p(_ptr(pos)), C.c_void_p(_ptr(u)),
                                                 C.c_void_p(_ptr(idp)) if idp is not None else None,
                                                 pos.shape[0], tau0, 1), "pm_init_particles")
        else:
            pos = np.ascontiguousarray(pos, dtype=np.float64)
            u = np.ascontiguousarray(u, dtype=self.np_dtype)
            idh = np.ascontiguousarray(ids, dtype=np.uint32) if ids is not None else None
            self._chk(self.lib.pm_init_particles(self.ctx, pos.ctypes.data, u.ctypes.data,
                                                 idh.ctypes.data if idh is not None else None,
                                                 pos.shape[0], tau0, 0), "pm_init_particles")

    def init_particles_2(self, pos, u, ids=None):
        """The second species (pm_init_particles_2): pos [n2][3] float64, u [n2][3] context precision,
        numpy (host) or CUDA tensors (device); after init_particles."""
        if isinstance(pos, torch.Tensor):
            pos = pos.to(torch.float64).contiguous()
            u = u.to(self.dtype).contiguous()
            idp = ids.to(torch.int32).contiguous() if ids is not None else None
            self._keep2 = (pos, u, idp)
            self._chk(self.lib.pm_init_particles_2(self.ctx, C.c_void_p(_ptr(pos)), C.c_void_p(_ptr(u)),
                                                   C.c_void_p(_ptr(idp)) if idp is not None else None,
                                                   pos.shape[0], 1), "pm_init_particles_2")
        else:
            pos = np.ascontiguousarray(pos, dtype=np.float64)
            u = np.ascontiguousarray(u, dtype=self.np_dtype)
            idh = np.ascontiguousarray(ids, dtype=np.uint32) if ids is not None else None
            self._chk(self.lib.pm_init_particles_2(self.ctx, pos.ctypes.data, u.ctypes.data,
                                                   idh.ctypes.data if idh is not None else None,
                                                   pos.shape[0], 0), "pm_init_particles_2")

    def get_particles_2(self):
        """(pos [n2][3] float64, u [n2][3]) of the second species in identifier order (host)."""
        pos = np.empty((self.np2, 3), dtype=np.float64)
        u = np.empty((self.np2, 3), dtype=self.np_dtype)
        self._chk(self.lib.pm_get_particles_2(self.ctx, pos.ctypes.data, u.ctypes.data, None, 0),
                  "pm_get_particles_2")
        return pos, u

    def deposit(self):
        self._chk(self.lib.pm_deposit(self.ctx), "pm_deposit")

    def solve_metric(self, dtau_prev: float):
        self._chk(self.lib.pm_solve_metric(self.ctx, dtau_prev), "pm_solve_metric")

    def update_particles(self, dtau: float):
        self._chk(self.lib.pm_update_particles(self.ctx, dtau), "pm_update_particles")

    def step(self, dtau: float):
        self._chk(self.lib.pm_step(self.ctx, dtau), "pm_step")

    # -- getters / setters -----------------------------------------------
    def get_field(self, name: str, device: bool = False):
        fid = L.FIELDS[name]
        if device:
            out = torch.empty((self.n,) * 3, dtype=self.dtype, device=self.device)
            self._chk(self.lib.pm_get_field(self.ctx, fid, C.c_void_p(_ptr(out)), 1), "pm_get_field")
            return out
        out = np.empty((self.n,) * 3, dtype=self.np_dtype)
        self._chk(self.lib.pm_get_field(self.ctx, fid, out.ctypes.data, 0), "pm_get_field")
        return out

    def set_field(self, name: str, arr):
        fid = L.FIELDS[name]
        if isinstance(arr, torch.Tensor):
            t = arr.to(device=self.device, dtype=self.dtype).contiguous()
            self._keep_field = t
            self._chk(self.lib.pm_set_field(self.ctx, fid, C.c_void_p(_ptr(t)), 1), "pm_set_field")
        else:
            a = np.ascontiguousarray(arr, dtype=self.np_dtype)
            assert a.size == self.n ** 3
            self._chk(self.lib.pm_set_field(self.ctx, fid, a.ctypes.data, 0), "pm_set_field")

    def get_particles(self, device: bool = False):
        """(pos [n][3] float64, u [n][3]) in identifier order."""
        if device:
            pos = torch.empty((self.np, 3), dtype=torch.float64, device=self.device)
            u = torch.empty((self.np, 3), dtype=self.dtype, device=self.device)
            self._chk(self.lib.pm_get_particles(self.ctx, C.c_void_p(_ptr(pos)), C.c_void_p(_ptr(u)), None, 1),
                      "pm_get_particles")
            return pos, u
        pos = np.empty((self.np, 3), dtype=np.float64)
        u = np.empty((self.np, 3), dtype=self.np_dtype)
        self._chk(self.lib.pm_get_particles(self.ctx, pos.ctypes.data, u.ctypes.data, None, 0), "pm_get_particles")
        return pos, u

    def diagnostics(self) -> dict:
        """pm_diagnostics: FP64 energy sum of the last deposit, mean phi of the last solve, total momentum."""
        out = (C.c_double * 5)()
        self._chk(self.lib.pm_diagnostics(self.ctx, out, 5), "pm_diagnostics")
        return {"energy_sum": out[0], "phi_mean": out[1], "momentum": (out[2], out[3], out[4])}

    def time(self):
        tau, a, steps = C.c_double(), C.c_double(), C.c_int64()
        self._chk(self.lib.pm_get_time(self.ctx, C.byref(tau), C.byref(a), C.byref(steps)), "pm_get_time")
        return tau.value, a.value, steps.value

    def timings(self) -> dict:
        """{stage: (total device ms, calls)} since the previous call; resets the counters."""
        ms = (C.c_double * 8)()
        calls = (C.c_int64 * 8)()
        self._chk(self.lib.pm_get_timings(self.ctx, ms, calls, 8), "pm_get_timings")
        return {name: (ms[i], calls[i]) for i, name in enumerate(L.STAGES)}

    def sync(self):
        self._chk(self.lib.pm_sync(self.ctx), "pm_sync")

    def get_state(self, device: bool = False):
        """Checkpoint of the time-stepping state (pm_get_state): a uint8 numpy array, or a uint8
        device tensor when `device`."""
        nb = C.c_size_t(0)
        self._chk(self.lib.pm_get_state(self.ctx, None, C.byref(nb), 0), "pm_get_state")
        if device:
            blob = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
            self._chk(self.lib.pm_get_state(self.ctx, C.c_void_p(_ptr(blob)), C.byref(nb), 1), "pm_get_state")
            return blob
        blob = np.empty(nb.value, dtype=np.uint8)
        self._chk(self.lib.pm_get_state(self.ctx, blob.ctypes.data, C.byref(nb), 0), "pm_get_state")
        return blob

    def set_state(self, blob):
        """Restore a checkpoint taken by get_state on a context of the same configuration."""
        if isinstance(blob, torch.Tensor) and blob.device.type != "cpu":
            b = blob.contiguous()
            self._chk(self.lib.pm_set_state(self.ctx, C.c_void_p(_ptr(b)), b.numel(), 1), "pm_set_state")
            return
        a = np.ascontiguousarray(blob.cpu().numpy() if isinstance(blob, torch.Tensor) else blob, dtype=np.uint8)
        self._chk(self.lib.pm_set_state(self.ctx, a.ctypes.data, a.size, 0), "pm_set_state")

    def power_spectrum(self, subtract_shot_noise: bool = True):
        """Shell-averaged P(k) of the current particles on this mesh (pm_power_spectrum):
        (k [h/Mpc], P [(Mpc/h)^3], modes) for the non-empty shells b = 1 .. n/2."""
        nb = self.n // 2 + 1
        k = np.zeros(nb)
        p = np.zeros(nb)
        m = np.zeros(nb)
        self._chk(self.lib.pm_power_spectrum(self.ctx, int(bool(subtract_shot_noise)), k.ctypes.data, p.ctypes.data,
                                             m.ctypes.data), "pm_power_spectrum")
        good = m > 0
        return k[good], p[good], m[good]

    def debug_fft(self, x: torch.Tensor, direction: int) -> torch.Tensor:
        n = self.n
        if direction == 1:
            x = x.to(device=self.device, dtype=self.dtype).contiguous()
            cdt = torch.complex128 if self.precision == "fp64" else torch.complex64
            out = torch.empty((n, n, n // 2 + 1), dtype=cdt, device=self.device)
        else:
            cdt = torch.complex128 if self.precision == "fp64" else torch.complex64
            x = x.to(device=self.device, dtype=cdt).contiguous()
            out = torch.empty((n, n, n), dtype=self.dtype, device=self.device)
        self._chk(self.lib.pm_debug_fft(self.ctx, C.c_void_p(_ptr(x)), C.c_void_p(_ptr(out)), direction),
                  "pm_debug_fft")
        return out

    # -- gathered force and the learned closure ---------------------------------
    def gather_grad_phi(self) -> torch.Tensor:
        """grad phi at the particles as the kick sees it, [n][3] in identifier order (device)."""
        out = torch.empty((self.np, 3), dtype=self.dtype, device=self.device)
        self._chk(self.lib.pm_gather_grad_phi(self.ctx, C.c_void_p(_ptr(out)), 1), "pm_gather_grad_phi")
        return out

    def closure_set_params(self, params, host: bool = False):
        """Bind the network's FP32 parameter vector; `host` passes it from host memory (src_on_device 0)."""
        if host:
            a = np.ascontiguousarray(params.cpu().numpy() if isinstance(params, torch.Tensor) else params,
                                     dtype=np.float32)
            assert a.size == L.PM_CLOSURE_NPARAM
            self._chk(self.lib.pm_closure_set_params(self.ctx, a.ctypes.data, 0), "pm_closure_set_params")
            return
        t = torch.as_tensor(params, dtype=torch.float32).to(self.device).contiguous()
        assert t.numel() == L.PM_CLOSURE_NPARAM
        self._keep_params = t
        self._chk(self.lib.pm_closure_set_params(self.ctx, C.c_void_p(_ptr(t)), 1), "pm_closure_set_params")

    def closure_enable(self, on: bool = True):
        self._chk(self.lib.pm_closure_enable(self.ctx, 1 if on else 0), "pm_closure_enable")

    def closure_forward(self, scaled: bool = False):
        self._chk(self.lib.pm_closure_forward(self.ctx, 1 if scaled else 0), "pm_closure_forward")

    def closure_gather(self) -> torch.Tensor:
        out = torch.empty((self.np, 3), dtype=torch.float32, device=self.device)
        self._chk(self.lib.pm_closure_gather(self.ctx, C.c_void_p(_ptr(out)), 1), "pm_closure_gather")
        return out

    def closure_backward(self, dpred: torch.Tensor) -> torch.Tensor:
        d = dpred.to(device=self.device, dtype=torch.float32).contiguous()
        g = torch.empty(L.PM_CLOSURE_NPARAM, dtype=torch.float32, device=self.device)
        self._chk(self.lib.pm_closure_backward(self.ctx, C.c_void_p(_ptr(d)), C.c_void_p(_ptr(g))),
                  "pm_closure_backward")
        return g

    def closure_loss(self, target: torch.Tensor, dpred: torch.Tensor | None = None, read: bool = True):
        """Residual of the last forward pass against target ([n][3] FP32, identifier order): returns
        (mean |pred - target|^2, mean |target|^2, dpred) with dpred the MSE gradient that
        closure_backward takes (written into `dpred` when given); with read=False the two means stay on
        the device and are returned as None (no synchronisation)."""
        t = target.to(device=self.device, dtype=torch.float32).contiguous()
        assert t.shape == (self.np, 3)
        if dpred is None:
            dpred = torch.empty((self.np, 3), dtype=torch.float32, device=self.device)
        assert dpred.is_cuda and dpred.dtype == torch.float32 and dpred.is_contiguous() and dpred.shape == (self.np, 3)
        out = (C.c_double * 2)()
        self._chk(self.lib.pm_closure_loss(self.ctx, C.c_void_p(_ptr(t)), C.c_void_p(_ptr(dpred)),
                                           out if read else None), "pm_closure_loss")
        return (out[0], out[1], dpred) if read else (None, None, dpred)

    def cube_symmetry(self, pos: torch.Tensor, u: torch.Tensor, v: torch.Tensor, perm, flip: int, out=None):
        """One of the 48 symmetries of the periodic cube on [n][3] device arrays (positions FP64, two FP32 vector
        fields): component d of the result is component perm[d] of the input; where bit d of flip is set the
        position is reflected (x -> 1 - x) and both vectors are negated.  Returns (pos, u, v); `out` may be the
        inputs themselves."""
        for t, dt in ((pos, torch.float64), (u, torch.float32), (v, torch.float32)):
            assert t.is_cuda and t.dtype == dt and t.is_contiguous() and t.dim() == 2 and t.shape[1] == 3
        n = pos.shape[0]
        assert u.shape[0] == n and v.shape[0] == n
        if out is None:
            out = (torch.empty_like(pos), torch.empty_like(u), torch.empty_like(v))
        p3 = (C.c_int * 3)(*[int(q) for q in perm])
        self._chk(self.lib.pm_cube_symmetry(self.ctx, n, p3, int(flip), *(C.c_void_p(_ptr(t)) for t in (pos, u, v)),
                                            *(C.c_void_p(_ptr(t)) for t in out)), "pm_cube_symmetry")
        return out

    def closure_adam(self, params: torch.Tensor, m: torch.Tensor, v: torch.Tensor, grad: torch.Tensor, step: int,
                     lr: float):
        for t in (params, m, v, grad):
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == L.PM_CLOSURE_NPARAM
        self._chk(self.lib.pm_closure_adam(self.ctx, C.c_void_p(_ptr(params)), C.c_void_p(_ptr(m)),
                                           C.c_void_p(_ptr(v)), C.c_void_p(_ptr(grad)), step, lr), "pm_closure_adam")

    def closure_scale(self) -> float:
        r = C.c_double()
        self._chk(self.lib.pm_closure_scale(self.ctx, C.byref(r)), "pm_closure_scale")
        return r.value
