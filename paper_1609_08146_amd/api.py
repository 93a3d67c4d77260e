"""Thin Python binding of the C ABI (include/sc.h).

Arguments are marshalled to the library; all computation runs in the gfx950
kernels of libsc.so.  Host arrays are numpy; device arrays are torch tensors
on the context's device (torch provides device memory and the stream only).
"""
from __future__ import annotations

import atexit
import ctypes
import weakref
from typing import Optional, Sequence

import numpy as np

from . import _abi
from ._abi import SC_FP32, SC_FP32_SPLIT, SC_FP64, ScError, call, call_status

PRECISIONS = {"fp64": SC_FP64, "fp32_split": SC_FP32_SPLIT, "fp32": SC_FP32}

_LIVE_CONTEXTS = weakref.WeakSet()


@atexit.register
def _close_all():
    # release device objects before the HIP runtime is torn down at process exit
    for c in list(_LIVE_CONTEXTS):
        try:
            c.close()
        except Exception:
            pass


def _prec(p) -> int:
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


def _host_f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _host_c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


_BEAMS = {"linear": 0, "radial": 1, "azimuthal": 2}


def _beam(b) -> int:
    return _BEAMS[b] if isinstance(b, str) else int(b)


def _ptr(a) -> int:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    # torch tensor
    assert a.is_contiguous(), "device tensors must be contiguous"
    return a.data_ptr()


def _is_device(a) -> bool:
    return a is not None and not isinstance(a, np.ndarray)


def _check_device(t, dtype: str, numel: int, what: str):
    """The library writes or reads `numel` elements through a raw pointer: check the tensor first."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what}: expected a torch tensor on the device")
    if t.dtype != getattr(torch, dtype):
        raise TypeError(f"{what}: expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: device tensors must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{what}: needs {numel} elements, got {t.numel()}")


def _check_host(a: np.ndarray, numel: int, what: str):
    if a.size != numel:
        raise ValueError(f"{what}: expected {numel} elements, got {a.size}")


class Context:
    """sc_ctx: one HIP device + stream.  stream=None uses torch's current stream on `device`."""

    def __init__(self, device: int = 0, stream=None, use_torch_stream: bool = True):
        self.device = device
        handle = None
        if stream is not None:
            handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        elif use_torch_stream:
            import torch
            handle = torch.cuda.current_stream(device).cuda_stream
        out = ctypes.c_void_p()
        call("sc_ctx_create", int(device), handle, ctypes.byref(out))
        self.h = out
        self._probs = weakref.WeakSet()
        self._servers = weakref.WeakSet()
        _LIVE_CONTEXTS.add(self)

    def close(self):
        """Destroy the context, closing every problem still open on it first."""
        if self.h:
            for sv in list(self._servers):
                sv.close()
            for p in list(self._probs):
                p.close()
            call("sc_ctx_destroy", self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def synchronize(self):
        call("sc_ctx_synchronize", self.h)

    def set_profiling(self, on: bool = True):
        call("sc_ctx_set_profiling", self.h, int(bool(on)))

    def evaluate_batch(self, probs: Sequence["Problem"], precision="fp32_split"):
        arr = (ctypes.c_void_p * len(probs))(*[p.h for p in probs])
        call("sc_evaluate_batch", self.h, arr, len(probs), _prec(precision))
        for p in probs:
            p._res_prec = _prec(precision)

    def set_batch_launch(self, precision="fp32_split", obs_per_lane=0, waves_per_block=0, chunk=0, blocks_per_cu=0,
                         freq_per_lane=0, reset=False):
        """Launch of evaluate_batch in `precision` (sc_set_batch_launch); reset=True clears it."""
        if reset:
            call("sc_set_batch_launch", self.h, _prec(precision), None)
            return
        l = _abi.sc_launch(obs_per_lane, waves_per_block, chunk, blocks_per_cu, freq_per_lane)
        call("sc_set_batch_launch", self.h, _prec(precision), ctypes.byref(l))

    def autotune_batch(self, probs: Sequence["Problem"], precision="fp32_split", budget_ms: float = 0.0) -> dict:
        """Tune the batched launch on `probs` (sc_autotune_batch); returns the winner."""
        arr = (ctypes.c_void_p * len(probs))(*[p.h for p in probs])
        l = _abi.sc_launch()
        call("sc_autotune_batch", self.h, arr, len(probs), _prec(precision), float(budget_ms), ctypes.byref(l))
        return {f: getattr(l, f) for f, _ in l._fields_}

    def autotune_save(self, path: str):
        call("sc_autotune_save", self.h, path.encode())

    def autotune_load(self, path: str):
        call("sc_autotune_load", self.h, path.encode())


class Problem:
    """sc_prob: one mirror, spectrum, incident field and observation set."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        if not ctx.h:
            raise ValueError("context is closed")
        out = ctypes.c_void_p()
        call("sc_prob_create", ctx.h, ctypes.byref(out))
        self.h = out
        ctx._probs.add(self)
        self.n_k = 0
        self.n_obs = 0
        self._res_prec = None

    def close(self):
        if self.h:
            if self.ctx.h:
                call("sc_prob_destroy", self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- inputs
    def set_mirror(self, f: float, r_max: float, n_r: int, n_phi: int):
        call("sc_set_mirror", self.h, float(f), float(r_max), int(n_r), int(n_phi))
        self.n_r, self.n_phi = int(n_r), int(n_phi)

    def set_surface(self, xyz, ndS, rim_xyz=None, rim_n=None, rim_dl=None):
        """A general mirror from its quadrature (sc_set_surface): nodes, n dS, and the oriented boundary."""
        xyz, ndS = _host_f64(xyz, (-1, 3)), _host_f64(ndS, (-1, 3))
        n_rim = 0 if rim_xyz is None else int(np.asarray(rim_xyz).reshape(-1, 3).shape[0])
        rx = rn = rdl = None
        if n_rim:
            rx, rn, rdl = _host_f64(rim_xyz, (-1, 3)), _host_f64(rim_n, (-1, 3)), _host_f64(rim_dl, (-1, 3))
            if rn.shape[0] != n_rim or rdl.shape[0] != n_rim:
                raise ValueError("rim arrays must have the same length")
        if ndS.shape != xyz.shape:
            raise ValueError("xyz and ndS must have the same shape")
        call("sc_set_surface", self.h, int(xyz.shape[0]), _ptr(xyz), _ptr(ndS), n_rim, _ptr(rx), _ptr(rn), _ptr(rdl))

    def num_nodes(self):
        ns, nr = ctypes.c_int(), ctypes.c_int()
        call("sc_get_num_nodes", self.h, ctypes.byref(ns), ctypes.byref(nr))
        return ns.value, nr.value

    def get_nodes(self):
        ns, nr = self.num_nodes()
        n = ns + nr
        xyz, nrm, w = np.empty((n, 3)), np.empty((n, 3)), np.empty(n)
        call("sc_get_nodes", self.h, _ptr(xyz), _ptr(nrm), _ptr(w))
        return xyz, nrm, w

    def set_frequencies(self, k):
        k = _host_f64(k).ravel()
        call("sc_set_frequencies", self.h, _ptr(k), int(k.shape[0]))
        self.n_k = int(k.shape[0])

    def set_incident(self, E, B):
        """E, B: complex128 [n_k][n_nodes_total][3] (numpy, or complex128 torch tensors on the device)."""
        dev = _is_device(E)
        ns, nr = self.num_nodes()
        numel = self.n_k * (ns + nr) * 3
        if dev:
            _check_device(E, "complex128", numel, "set_incident E")
            _check_device(B, "complex128", numel, "set_incident B")
        else:
            E, B = _host_c128(E), _host_c128(B)
            _check_host(E, numel, "set_incident E")
            _check_host(B, numel, "set_incident B")
        call("sc_set_incident", self.h, _ptr(E), _ptr(B), int(dev))

    def set_incident_gaussian(self, w0: float, pol: float = 0.0, spectrum=None, consistent: bool = False):
        sp = None if spectrum is None else _host_c128(spectrum).ravel()
        call("sc_set_incident_gaussian", self.h, float(w0), float(pol), _ptr(sp), int(bool(consistent)))

    def set_incident_beam(self, beam, w0: float, pol: float = 0.0, spectrum=None, consistent: bool = False):
        """beam: 0/'linear', 1/'radial', 2/'azimuthal' (sc_set_incident_beam)."""
        sp = None if spectrum is None else _host_c128(spectrum).ravel()
        call("sc_set_incident_beam", self.h, _beam(beam), float(w0), float(pol), _ptr(sp), int(bool(consistent)))

    def set_incident_lg(self, modes, w0: float, spectrum=None):
        """Laguerre-Gauss mode set (sc_set_incident_lg): modes is a sequence of (p, l, ex, ey) with
        complex amplitudes ex, ey of the x- and y-polarised parts."""
        arr = (_abi.sc_lg_mode * len(modes))()
        for i, (pp, ll, ex, ey) in enumerate(modes):
            arr[i].p, arr[i].l = int(pp), int(ll)
            arr[i].ex[0], arr[i].ex[1] = float(np.real(ex)), float(np.imag(ex))
            arr[i].ey[0], arr[i].ey[1] = float(np.real(ey)), float(np.imag(ey))
        sp = None if spectrum is None else _host_c128(spectrum).ravel()
        call("sc_set_incident_lg", self.h, arr, len(modes), float(w0), _ptr(sp))

    def incident_power(self):
        """Power of each frequency component through the aperture, [n_k] (sc_get_incident_power)."""
        P = np.empty(self.n_k, np.float64)
        call("sc_get_incident_power", self.h, _ptr(P))
        return P

    def scale_spectrum(self, factor):
        """Multiply frequency n of the incident field by factor[n] (complex)."""
        f = _host_c128(factor).ravel()
        if f.shape[0] != self.n_k:
            raise ValueError(f"factor has {f.shape[0]} entries, expected {self.n_k}")
        call("sc_scale_spectrum", self.h, _ptr(f))

    def normalize_energy(self, eps, e_tot: float = 0.0, dk: float = 0.0):
        """Scale the spectrum to the power spectrum eps (optionally normalised to e_tot)."""
        e = _host_f64(eps, (-1,))
        if e.shape[0] != self.n_k:
            raise ValueError(f"eps has {e.shape[0]} entries, expected {self.n_k}")
        call("sc_normalize_energy", self.h, _ptr(e), float(e_tot), float(dk))

    # ---- diagnostics (the observation set must be the 13-point stencils of n_pts points)
    def maxwell_residual_freq(self, n_pts: int, h: float):
        """|e_f| [n_k][n_pts] from the last result (sc_maxwell_residual_freq)."""
        out = np.empty((self.n_k, n_pts), np.float64)
        call("sc_maxwell_residual_freq", self.h, int(n_pts), float(h), _ptr(out))
        return out

    def maxwell_residual_time(self, n_pts: int, h: float, t, dt: float, dk: float):
        """|e_t| [n_t][n_pts] from the last result (sc_maxwell_residual_time)."""
        t = _host_f64(t, (-1,))
        out = np.empty((t.shape[0], n_pts), np.float64)
        call("sc_maxwell_residual_time", self.h, int(n_pts), float(h), _ptr(t), int(t.shape[0]), float(dt),
             float(dk), _ptr(out))
        return out

    def field_energy(self, t, dk: float, dV: float):
        """Energy of the observation set at times t [n_t] (sc_field_energy)."""
        t = _host_f64(t, (-1,))
        out = np.empty(t.shape[0], np.float64)
        call("sc_field_energy", self.h, _ptr(t), int(t.shape[0]), float(dk), float(dV), _ptr(out))
        return out

    def set_table_storage(self, keep_fp64: bool):
        call("sc_set_table_storage", self.h, int(bool(keep_fp64)))

    def set_factoring(self, enable: bool, tie_charge: bool = True):
        """Use the factored current J~ = u s for "fp32_split" and "fp64" when the tables allow it,
        and with `tie_charge` the charge tied to it, rho~ = -i beta s / k, where it is
        (sc_set_factoring with 1; 2 without the tied charge, 0 neither)."""
        call("sc_set_factoring", self.h, 0 if not enable else (1 if tie_charge else 2))

    @property
    def factored(self) -> bool:
        """True if "fp32_split" evaluation uses the factored tables (sc_get_factoring)."""
        v = ctypes.c_int(0)
        call("sc_get_factoring", self.h, ctypes.byref(v))
        return bool(v.value)

    def factored_for(self, precision="fp32_split") -> bool:
        """True if evaluation in `precision` uses the factored tables (sc_get_factoring_for)."""
        return self.layout_for(precision) != "general"

    def layout_for(self, precision="fp32_split") -> str:
        """Table layout of evaluation in `precision`: "general", "factored" (the current J~ = u s)
        or "tied" (the factored current and the charge tied to it), from sc_get_factoring_for."""
        v = ctypes.c_int(0)
        call("sc_get_factoring_for", self.h, _prec(precision), ctypes.byref(v))
        return ("general", "factored", "tied")[v.value]

    def set_observation(self, xyz):
        dev = _is_device(xyz)
        if not dev:
            xyz = _host_f64(xyz, (-1, 3))
        elif xyz.dim() != 2 or xyz.shape[1] != 3:
            raise ValueError("set_observation: device points must have shape [n, 3]")
        else:
            _check_device(xyz, "float64", 3 * xyz.shape[0], "set_observation")
        n = int(xyz.shape[0])
        call("sc_set_observation", self.h, _ptr(xyz), n, int(dev))
        self.n_obs = n

    def set_launch(self, obs_per_lane=0, waves_per_block=0, chunk=0, blocks_per_cu=0, freq_per_lane=0,
                   reset=False):
        if reset:
            call("sc_set_launch", self.h, None)
            return
        l = _abi.sc_launch(obs_per_lane, waves_per_block, chunk, blocks_per_cu, freq_per_lane)
        call("sc_set_launch", self.h, ctypes.byref(l))

    def launch(self, precision="fp32_split") -> dict:
        """The launch shape an evaluation in `precision` uses now (sc_get_launch)."""
        l = _abi.sc_launch()
        call("sc_get_launch", self.h, _prec(precision), ctypes.byref(l))
        return {f: getattr(l, f) for f, _ in l._fields_}

    def autotune(self, precision="fp32_split", budget_ms: float = 0.0):
        l = _abi.sc_launch()
        call("sc_autotune", self.h, _prec(precision), float(budget_ms), ctypes.byref(l))
        return dict(obs_per_lane=l.obs_per_lane, waves_per_block=l.waves_per_block, chunk=l.chunk,
                    blocks_per_cu=l.blocks_per_cu, freq_per_lane=l.freq_per_lane)

    # ---- evaluation
    def _out_host(self, prec, n_first):
        dt = np.complex128 if prec == SC_FP64 else np.complex64
        return np.empty((n_first, self.n_obs, 3), dt)

    def evaluate(self, precision="fp32_split", out=None, keep_on_device: bool = False):
        """Evaluate; returns host (E, B) arrays [n_k][n_obs][3], or fills `out`=(E, B) device tensors."""
        prec = _prec(precision)
        self._res_prec = prec
        if keep_on_device:
            call("sc_evaluate", self.h, prec, None, None, 1)
            return None
        if out is not None:
            E, B = out
            dt = "complex128" if prec == SC_FP64 else "complex64"
            for t, name in ((E, "evaluate E"), (B, "evaluate B")):
                _check_device(t, dt, self.n_k * self.n_obs * 3, name)
            call("sc_evaluate", self.h, prec, _ptr(E), _ptr(B), 1)
            return out
        E, B = self._out_host(prec, self.n_k), self._out_host(prec, self.n_k)
        call("sc_evaluate", self.h, prec, _ptr(E), _ptr(B), 0)
        return E, B

    def evaluate_noalloc(self, out, precision="fp32_split"):
        """sc_evaluate_noalloc: evaluate into device tensors out=(E, B) without any allocation (the
        problem must have been evaluated once in this precision; the stored result is unchanged)."""
        prec = _prec(precision)
        E, B = out
        dt = "complex128" if prec == SC_FP64 else "complex64"
        for t, name in ((E, "evaluate_noalloc E"), (B, "evaluate_noalloc B")):
            _check_device(t, dt, self.n_k * self.n_obs * 3, name)
        call("sc_evaluate_noalloc", self.h, prec, _ptr(E), _ptr(B))
        return out

    def result(self):
        E, B = self._out_host(self._res_prec, self.n_k), self._out_host(self._res_prec, self.n_k)
        call("sc_get_result", self.h, _ptr(E), _ptr(B), 0)
        return E, B

    def _time_out(self, n_t, out, name):
        if out is not None:
            Et, Bt = out
            dt = "complex128" if self._res_prec == SC_FP64 else "complex64"
            for a, nm in ((Et, f"{name} Et"), (Bt, f"{name} Bt")):
                _check_device(a, dt, n_t * self.n_obs * 3, nm)
            return Et, Bt, 1
        return self._out_host(self._res_prec, n_t), self._out_host(self._res_prec, n_t), 0

    def to_time(self, t0: float, dt: float, n_t: int, out=None):
        """sc_to_time: the last result at times t0 + m dt, m < n_t, with dk the step of the uniform
        frequency grid; host arrays [n_t][n_obs][3], or fills `out`=(Et, Bt) device tensors."""
        Et, Bt, dev = self._time_out(int(n_t), out, "to_time")
        call("sc_to_time", self.h, float(t0), float(dt), int(n_t), _ptr(Et), _ptr(Bt), dev)
        return Et, Bt

    def to_time_at(self, dk: float, t, out=None):
        """sc_to_time_at: the last result at the times t[] with the frequency weight dk."""
        t = _host_f64(t).ravel()
        Et, Bt, dev = self._time_out(t.shape[0], out, "to_time_at")
        call("sc_to_time_at", self.h, float(dk), _ptr(t), int(t.shape[0]), _ptr(Et), _ptr(Bt), dev)
        return Et, Bt

    def timing(self) -> dict:
        tm = _abi.sc_timing()
        call("sc_get_timing", self.h, ctypes.byref(tm))
        return {f: getattr(tm, f) for f, _ in tm._fields_}

    def device_bytes(self) -> int:
        b = ctypes.c_size_t()
        call("sc_prob_device_bytes", self.h, ctypes.byref(b))
        return b.value


def stencil_points(xyz, h: float) -> np.ndarray:
    """The 13-point finite-difference stencils of points xyz [n, 3] (sc_stencil_points), [13 n, 3]."""
    xyz = _host_f64(xyz, (-1, 3))
    out = np.empty((13 * xyz.shape[0], 3), np.float64)
    call("sc_stencil_points", _ptr(xyz), int(xyz.shape[0]), float(h), _ptr(out))
    return out


def problem_from_workload(ctx: Context, w, consistent: Optional[bool] = None) -> Problem:
    """A Problem set up with a ``workloads.Workload``'s mirror, spectrum, Gaussian beam and points."""
    p = Problem(ctx)
    p.set_mirror(w.f, w.a, w.n_r, w.n_phi)
    p.set_frequencies(w.k)
    p.set_incident_beam(getattr(w, "beam", 0), w.w0, w.pol, w.spectrum,
                        bool(w.consistent if consistent is None else consistent))
    p.set_observation(w.obs)
    return p


class Server:
    """sc_server: continuous-batching serving loop on a context (thread-safe submit / wait)."""

    def __init__(self, ctx: Context, hbm_budget: int, max_running: int = 8, quantum_ms: float = 20.0):
        self.ctx = ctx
        out = ctypes.c_void_p()
        call("sc_server_create", ctx.h, ctypes.c_size_t(int(hbm_budget)), int(max_running), float(quantum_ms),
             ctypes.byref(out))
        self.h = out
        self._meta = {}
        ctx._servers.add(self)

    def close(self):
        if self.h:
            if self.ctx.h:
                call("sc_server_destroy", self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, w, precision="fp32_split", t=None, dk: float = 1.0, consistent: Optional[bool] = None) -> int:
        """Queue a solve of a ``workloads.Workload``; returns its ticket."""
        k = _host_f64(w.k).ravel()
        spec = None if w.spectrum is None else _host_c128(w.spectrum).ravel()
        obs = _host_f64(w.obs, (-1, 3))
        tt = None if t is None else _host_f64(t).ravel()
        req = _abi.sc_request(
            f=float(w.f), r_max=float(w.a), n_r=int(w.n_r), n_phi=int(w.n_phi), n_k=int(k.shape[0]),
            k=_ptr(k), spectrum=_ptr(spec), w0=float(w.w0), pol_angle=float(w.pol),
            consistent=int(bool(w.consistent if consistent is None else consistent)), n_obs=int(obs.shape[0]),
            obs=_ptr(obs), prec=_prec(precision), n_t=0 if tt is None else int(tt.shape[0]), t=_ptr(tt),
            dk=float(dk), beam=_beam(getattr(w, "beam", 0)))
        ticket = ctypes.c_uint64()
        call("sc_server_submit", self.h, ctypes.byref(req), ctypes.byref(ticket))
        self._meta[ticket.value] = (_prec(precision), int(k.shape[0]), int(obs.shape[0]),
                                    0 if tt is None else int(tt.shape[0]))
        return ticket.value

    def wait(self, ticket: int, timeout_ms: float = -1.0):
        """Block for a result: (E, B, Et, Bt, stats) on the host (Et, Bt None without time samples)."""
        prec, n_k, n_obs, n_t = self._meta[ticket]
        dt = np.complex128 if prec == SC_FP64 else np.complex64
        E, B = np.empty((n_k, n_obs, 3), dt), np.empty((n_k, n_obs, 3), dt)
        Et = Bt = None
        if n_t:
            Et, Bt = np.empty((n_t, n_obs, 3), dt), np.empty((n_t, n_obs, 3), dt)
        st = _abi.sc_request_stats()
        call("sc_server_wait", self.h, ctypes.c_uint64(ticket), float(timeout_ms), _ptr(E), _ptr(B), _ptr(Et),
             _ptr(Bt), ctypes.byref(st))
        self._meta.pop(ticket, None)
        stats = {f: getattr(st, f) for f, _ in st._fields_}
        return E, B, Et, Bt, stats

    def wait_status(self, ticket: int, timeout_ms: float = -1.0) -> int:
        """Wait and return only the status code (the result, if any, is discarded)."""
        prec, n_k, n_obs, n_t = self._meta[ticket]
        st = call_status("sc_server_wait", self.h, ctypes.c_uint64(ticket), float(timeout_ms), None, None, None,
                         None, None)
        if st not in (_abi.SC_E_TIMEOUT,):
            self._meta.pop(ticket, None)
        return st

    def cancel(self, ticket: int):
        call("sc_server_cancel", self.h, ctypes.c_uint64(ticket))

    def stats(self) -> dict:
        s = _abi.sc_server_stats()
        call("sc_server_get_stats", self.h, ctypes.byref(s))
        return {f: getattr(s, f) for f, _ in s._fields_}
