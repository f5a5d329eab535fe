"""ctypes binding of libvlb.so (C ABI in include/vlb.h).  Argument marshalling only.

PyTorch supplies the device memory (one uint8 workspace tensor bound to each batch)
and the HIP stream (torch's current stream); every numerical step runs in the
library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
VLB_FP64, VLB_MIXED = 0, 1
VLB_TAU_AOKI, VLB_TAU_HYDRO, VLB_TAU_KN = 0, 1, 2

_lib = None


def library_path() -> str:
    return os.path.join(HERE, "libvlb.so")


class VlbError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status} ({message})")
        self.status = status


class _Axis(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("Q", ctypes.c_int), ("N", ctypes.c_int)]


class _CouetteDesc(ctypes.Structure):
    _fields_ = [("R_in", ctypes.c_double), ("R_out", ctypes.c_double), ("N_R", ctypes.c_int),
                ("A", ctypes.c_double), ("delta", ctypes.c_double), ("ax1", _Axis), ("ax2", _Axis),
                ("Kn", ctypes.c_double), ("tau_model", ctypes.c_int), ("dt", ctypes.c_double),
                ("cfl", ctypes.c_double), ("u_in", ctypes.c_double), ("T_in", ctypes.c_double),
                ("u_out", ctypes.c_double), ("T_out", ctypes.c_double), ("weno_eps", ctypes.c_double),
                ("form", ctypes.c_int)]


@dataclass
class CouetteDesc:
    """One circular-Couette instance; ax1 / ax2 = (kind, Q, N) with kind 0 = full range
    H(N;Q), 1 = half range HH(N;Q)."""
    R_in: float = 1.0
    R_out: float = 2.0
    N_R: int = 64
    ax1: tuple = (1, 4, 2)
    ax2: tuple = (0, 4, 2)
    Kn: float = 0.1
    tau_model: int = VLB_TAU_AOKI
    dt: float = 0.0
    cfl: float = 0.5
    u_in: float = 0.1
    T_in: float = 1.0
    u_out: float = 0.0
    T_out: float = 1.0
    A: float = 0.0
    delta: float = 0.5
    weno_eps: float = 0.0
    form: int = 0             # 0: chi formulation; 1: f-tilde formulation (comparison only, FP64)

    def _c(self) -> _CouetteDesc:
        return _CouetteDesc(self.R_in, self.R_out, self.N_R, self.A, self.delta, _Axis(*self.ax1),
                            _Axis(*self.ax2), self.Kn, self.tau_model, self.dt, self.cfl, self.u_in,
                            self.T_in, self.u_out, self.T_out, self.weno_eps, self.form)


_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)


class _ChannelDesc(ctypes.Structure):
    _fields_ = [("N_lambda", ctypes.c_int), ("N_xi", ctypes.c_int), ("xi_in", ctypes.c_double),
                ("xi_out", ctypes.c_double), ("r", ctypes.c_double), ("L", ctypes.c_double), ("ax1", _Axis),
                ("ax2", _Axis), ("Kn", ctypes.c_double), ("tau_model", ctypes.c_int), ("dt", ctypes.c_double),
                ("cfl", ctypes.c_double), ("n_in", ctypes.c_double), ("n_out", ctypes.c_double),
                ("T_w", ctypes.c_double), ("weno_eps", ctypes.c_double),
                ("half", ctypes.c_int), ("ends", ctypes.c_int), ("Q0", ctypes.c_double),
                ("cartesian", ctypes.c_int), ("A", ctypes.c_double), ("kernel", ctypes.c_int)]


@dataclass
class ChannelDesc:
    """One expanding channel: N_lambda x N_xi cells, lambda in [-1, 1], xi in
    [xi_in, xi_out], wall 1 + phi(xi) with expansion ratio r over length L; ax1 (p^lambda,
    half range) and ax2 (p^xi) as (kind, Q, N); reservoir densities n_in / n_out; half:
    lambda in [0, 1] with a specular centreline; ends = 1: flow-rate profile of Q0."""
    N_lambda: int = 8
    N_xi: int = 12
    xi_in: float = -4.0
    xi_out: float = 12.0
    r: float = 2.0
    L: float = 4.0
    ax1: tuple = (1, 4, 2)
    ax2: tuple = (0, 4, 2)
    Kn: float = 0.05
    tau_model: int = 1
    dt: float = 0.0
    cfl: float = 0.5
    n_in: float = 1.1
    n_out: float = 0.9
    T_w: float = 1.0
    weno_eps: float = 0.0
    half: bool = False
    ends: int = 0
    Q0: float = 0.0
    cartesian: bool = False   # Cartesian-split momentum space (Sec. VI.G)
    A: float = 0.0            # lambda stretching towards the walls (Eq. canalie_stretch); 0 = equal cells
    kernel: int = 0           # 0 automatic, 1 velocity tiles (matrix cores), 2 population kernel (FP64)

    def _c(self) -> _ChannelDesc:
        return _ChannelDesc(self.N_lambda, self.N_xi, self.xi_in, self.xi_out, self.r, self.L, _Axis(*self.ax1),
                            _Axis(*self.ax2), self.Kn, self.tau_model, self.dt, self.cfl, self.n_in, self.n_out,
                            self.T_w, self.weno_eps, int(bool(self.half)), int(self.ends), float(self.Q0),
                            int(bool(self.cartesian)), float(self.A), int(self.kernel))
_SIGS = {
    "vlb_batch_create_couette": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(_CouetteDesc),
                                 ctypes.c_int, ctypes.c_void_p, ctypes.c_int],
    "vlb_batch_destroy": [ctypes.c_void_p],
    "vlb_batch_workspace_bytes": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "vlb_batch_bind_workspace": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t],
    "vlb_batch_info": [ctypes.c_void_p, ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 4
    + [_dp, ctypes.POINTER(ctypes.c_size_t)],
    "vlb_batch_state_size": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "vlb_batch_velocities": [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp, _dp],
    "vlb_set_wall": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double],
    "vlb_init_equilibrium": [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp, _dp],
    "vlb_set_state": [ctypes.c_void_p, _dp, ctypes.c_size_t],
    "vlb_get_state": [ctypes.c_void_p, _dp, ctypes.c_size_t],
    "vlb_step": [ctypes.c_void_p, ctypes.c_long],
    "vlb_step_fp64": [ctypes.c_void_p, ctypes.c_long],
    "vlb_mixed_fp32_steps": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_long)],
    "vlb_mixed_report": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "vlb_apply_L": [ctypes.c_void_p, _dp, ctypes.c_size_t],
    "vlb_moments": [ctypes.c_void_p, ctypes.c_int] + [_dp] * 7,
    "vlb_residual": [ctypes.c_void_p, _dp],
    "vlb_total_mass": [ctypes.c_void_p, _dp],
    "vlb_run_to_steady": [ctypes.c_void_p, ctypes.c_double, ctypes.c_long, ctypes.c_int,
                          ctypes.POINTER(ctypes.c_long), _dp],
    "vlb_axis_tables": [_Axis, _dp, _dp, _dp, _dp],
    "vlb_timing_enable": [ctypes.c_void_p, ctypes.c_int],
    "vlb_batch_set_graphs": [ctypes.c_void_p, ctypes.c_int],
    "vlb_batch_set_persistent": [ctypes.c_void_p, ctypes.c_int],
    "vlb_batch_set_tile": [ctypes.c_void_p, ctypes.c_int],
    "vlb_batch_get_tile": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)],
    "vlb_batch_autotune": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _dp],
    "vlb_timing_query": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                         ctypes.POINTER(ctypes.c_long), _dp, _dp],
    "vlb_mlp_param_count": [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
    "vlb_mlp_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int, _fp, ctypes.c_void_p],
    "vlb_mlp_destroy": [ctypes.c_void_p],
    "vlb_mlp_get_params": [ctypes.c_void_p, _fp, ctypes.c_size_t],
    "vlb_mlp_set_params": [ctypes.c_void_p, _fp, ctypes.c_size_t],
    "vlb_mlp_forward": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_long, ctypes.c_void_p, ctypes.c_int],
    "vlb_mlp_loss_grad": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_long, _fp, _fp],
    "vlb_mlp_adam_step": [ctypes.c_void_p, _fp, ctypes.c_float],
    "vlb_mlp_train": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_long,
                      ctypes.POINTER(ctypes.c_int), ctypes.c_long, ctypes.c_int, ctypes.c_float, _fp],
    "vlb_batch_surrogate_samples": [ctypes.c_void_p, _fp, _fp, ctypes.c_size_t],
    "vlb_batch_warm_start": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
    "vlb_batch_set_stall_window": [ctypes.c_void_p, ctypes.c_long],
    "vlb_batch_warm_report": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_long)],
    "vlb_channel_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(_ChannelDesc), ctypes.c_int,
                           ctypes.c_void_p],
    "vlb_channel_destroy": [ctypes.c_void_p],
    "vlb_channel_create_deferred": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(_ChannelDesc),
                                    ctypes.c_int, ctypes.c_void_p],
    "vlb_channel_workspace_bytes": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "vlb_channel_bind_workspace": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t],
    "vlb_channel_set_open_bc": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double],
    "vlb_channel_init_equilibrium": [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp, _dp],
    "vlb_channel_total_mass": [ctypes.c_void_p, _dp],
    "vlb_channel_last_run_seconds": [ctypes.c_void_p, _dp],
    "vlb_batch_last_run_seconds": [ctypes.c_void_p, _dp],
    "vlb_channel_info": [ctypes.c_void_p, ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 3
    + [_dp, ctypes.POINTER(ctypes.c_size_t)],
    "vlb_channel_state_size": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "vlb_channel_set_state": [ctypes.c_void_p, _dp, ctypes.c_size_t],
    "vlb_channel_get_state": [ctypes.c_void_p, _dp, ctypes.c_size_t],
    "vlb_channel_get_instance_state": [ctypes.c_void_p, ctypes.c_int, _dp, ctypes.c_size_t],
    "vlb_channel_set_instance_state": [ctypes.c_void_p, ctypes.c_int, _dp, ctypes.c_size_t],
    "vlb_channel_step": [ctypes.c_void_p, ctypes.c_long],
    "vlb_channel_step_fp64": [ctypes.c_void_p, ctypes.c_long],
    "vlb_channel_fp32_steps": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_long)],
    "vlb_channel_apply_L": [ctypes.c_void_p, _dp, ctypes.c_size_t],
    "vlb_channel_residual": [ctypes.c_void_p, _dp],
    "vlb_channel_moments": [ctypes.c_void_p, ctypes.c_int] + [_dp] * 5,
    "vlb_channel_flow_fields": [ctypes.c_void_p, ctypes.c_int] + [_dp] * 6,
    "vlb_channel_set_graphs": [ctypes.c_void_p, ctypes.c_int],
    "vlb_channel_run_to_steady": [ctypes.c_void_p, ctypes.c_double, ctypes.c_long, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_long), _dp],
    "vlb_couette_step_noalloc": [ctypes.c_int, ctypes.POINTER(_CouetteDesc), ctypes.c_void_p, ctypes.c_long, _dp,
                                 ctypes.c_void_p],
    "vlb_status_string": [ctypes.c_int],
    "vlb_last_error": [],
}


def load_library():
    """Load libvlb.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1708_05944_amd.build`")
    lib = ctypes.CDLL(path)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.vlb_status_string.restype = ctypes.c_char_p
    lib.vlb_last_error.restype = ctypes.c_char_p
    lib.vlb_batch_destroy.restype = None
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != 0:
        lib = load_library()
        raise VlbError(status, where, lib.vlb_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def axis_tables(kind: int, Q: int, N: int = 0):
    """Host tables of one axis as built by the library: (p, w, K, Kt)."""
    lib = load_library()
    n = Q if kind == 0 else 2 * Q
    p, w = np.zeros(n), np.zeros(n)
    K, Kt = np.zeros((n, n)), np.zeros((n, n))
    _check(lib.vlb_axis_tables(_Axis(kind, Q, N), _ptr(p), _ptr(w), _ptr(K), _ptr(Kt)), "vlb_axis_tables")
    return p, w, K, Kt


class Batch:
    """B Couette instances advanced together on one GPU."""

    def __init__(self, descs, precision: int = VLB_FP64, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the vielbein LB library runs on the GPU only")
        self._torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        lib = load_library()
        self.descs = list(descs)
        arr = (_CouetteDesc * len(self.descs))(*[d._c() for d in self.descs])
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(lib.vlb_batch_create_couette(ctypes.byref(h), len(self.descs), arr, precision,
                                            ctypes.c_void_p(self.stream.cuda_stream), 1), "vlb_batch_create_couette")
        self._h = h
        nbytes = ctypes.c_size_t()
        _check(lib.vlb_batch_workspace_bytes(h, ctypes.byref(nbytes)), "vlb_batch_workspace_bytes")
        self._ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        aligned = (base + 255) & ~255
        _check(lib.vlb_batch_bind_workspace(h, ctypes.c_void_p(aligned), nbytes.value), "vlb_batch_bind_workspace")
        self.B = len(self.descs)
        n = ctypes.c_size_t()
        _check(lib.vlb_batch_state_size(h, ctypes.byref(n)), "vlb_batch_state_size")
        self.state_size = n.value
        self.info = [self._info(b) for b in range(self.B)]

    def _info(self, b):
        lib = load_library()
        NR, NV, n1, n2 = (ctypes.c_int() for _ in range(4))
        dt = ctypes.c_double()
        off = ctypes.c_size_t()
        _check(lib.vlb_batch_info(self._h, b, ctypes.byref(NR), ctypes.byref(NV), ctypes.byref(n1), ctypes.byref(n2),
                                  ctypes.byref(dt), ctypes.byref(off)), "vlb_batch_info")
        return dict(N_R=NR.value, NV=NV.value, nodes1=n1.value, nodes2=n2.value, dt=dt.value, offset=off.value)

    def close(self):
        if getattr(self, "_h", None):
            load_library().vlb_batch_destroy(self._h)
            self._h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ state
    def instance_view(self, state: np.ndarray, b: int) -> np.ndarray:
        i = self.info[b]
        n = 2 * i["N_R"] * i["NV"]
        return state[i["offset"]:i["offset"] + n].reshape(2, i["N_R"], i["NV"])

    def get_state(self) -> np.ndarray:
        out = np.empty(self.state_size)
        _check(load_library().vlb_get_state(self._h, _ptr(out), out.size), "vlb_get_state")
        return out

    def set_state(self, state: np.ndarray):
        s = np.ascontiguousarray(state, dtype=np.float64).ravel()
        _check(load_library().vlb_set_state(self._h, _ptr(s), s.size), "vlb_set_state")

    def set_instance_state(self, b: int, F: np.ndarray):
        st = self.get_state()
        self.instance_view(st, b)[...] = F
        self.set_state(st)

    def init_equilibrium(self, b: int, n, u1, u2, T):
        cells = self.info[b]["N_R"] if b >= 0 else sum(i["N_R"] for i in self.info)
        arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(x, dtype=np.float64), (cells,))) for x in (n, u1, u2, T)]
        _check(load_library().vlb_init_equilibrium(self._h, b, *[_ptr(a) for a in arrs]), "vlb_init_equilibrium")

    def set_wall(self, b: int, side: int, u: float, T: float):
        _check(load_library().vlb_set_wall(self._h, b, side, u, T), "vlb_set_wall")

    # ------------------------------------------------------------------ stepping
    def step(self, nsteps: int = 1):
        _check(load_library().vlb_step(self._h, nsteps), "vlb_step")

    def step_fp64(self, nsteps: int = 1):
        _check(load_library().vlb_step_fp64(self._h, nsteps), "vlb_step_fp64")

    def fp32_steps(self) -> int:
        n = ctypes.c_long()
        _check(load_library().vlb_mixed_fp32_steps(self._h, ctypes.byref(n)), "vlb_mixed_fp32_steps")
        return n.value

    def last_run_seconds(self) -> float:
        """Wall-clock seconds of the last run_to_steady call."""
        s = ctypes.c_double()
        _check(load_library().vlb_batch_last_run_seconds(self._h, ctypes.byref(s)), "vlb_batch_last_run_seconds")
        return s.value

    def mixed_report(self):
        """Per instance: (relaxation factor of the defect correction, step at which it left
        the correction for FP64 steps for good or -1, FP32 correction steps taken)."""
        theta = np.empty(self.B)
        at = np.empty(self.B, dtype=np.int64)
        n32 = np.empty(self.B, dtype=np.int64)
        vp = ctypes.c_void_p
        _check(load_library().vlb_mixed_report(self._h, theta.ctypes.data_as(vp), at.ctypes.data_as(vp),
                                               n32.ctypes.data_as(vp)), "vlb_mixed_report")
        return theta, at, n32

    def apply_L(self) -> np.ndarray:
        out = np.empty(self.state_size)
        _check(load_library().vlb_apply_L(self._h, _ptr(out), out.size), "vlb_apply_L")
        return out

    def run_to_steady(self, tol: float, max_steps: int, check_every: int = 100):
        steps = (ctypes.c_long * self.B)()
        r = np.empty(self.B)
        st = load_library().vlb_run_to_steady(self._h, tol, max_steps, check_every, steps, _ptr(r))
        if st not in (0, -5):
            _check(st, "vlb_run_to_steady")
        return np.array(list(steps)), r, st == 0

    # ------------------------------------------------------------------ diagnostics
    def moments(self, b: int) -> dict:
        NR = self.info[b]["N_R"]
        outs = [np.empty(NR) for _ in range(7)]
        _check(load_library().vlb_moments(self._h, b, *[_ptr(o) for o in outs]), "vlb_moments")
        return dict(zip(("n", "u1", "u2", "T", "T12", "q1", "q2"), outs))

    def residual(self) -> np.ndarray:
        r = np.empty(self.B)
        _check(load_library().vlb_residual(self._h, _ptr(r)), "vlb_residual")
        return r

    def total_mass(self) -> np.ndarray:
        m = np.empty(self.B)
        _check(load_library().vlb_total_mass(self._h, _ptr(m)), "vlb_total_mass")
        return m

    def set_tile(self, cells_per_run: int):
        _check(load_library().vlb_batch_set_tile(self._h, cells_per_run), "vlb_batch_set_tile")

    def tile(self) -> int:
        t = ctypes.c_int()
        _check(load_library().vlb_batch_get_tile(self._h, ctypes.byref(t)), "vlb_batch_get_tile")
        return t.value

    def autotune(self, steps: int = 5):
        """Pick the cells-per-run of the stage kernel by timing; returns (tile, ms/step)."""
        t = ctypes.c_int()
        ms = ctypes.c_double()
        _check(load_library().vlb_batch_autotune(self._h, steps, ctypes.byref(t), ctypes.byref(ms)),
               "vlb_batch_autotune")
        return t.value, ms.value

    def set_graphs(self, on: bool = True):
        _check(load_library().vlb_batch_set_graphs(self._h, 1 if on else 0), "vlb_batch_set_graphs")

    def set_persistent(self, max_blocks: int = 64):
        """Multi-step cooperative launches for block lists of at most max_blocks blocks (0: off)."""
        _check(load_library().vlb_batch_set_persistent(self._h, max_blocks), "vlb_batch_set_persistent")

    def timing_enable(self, on: bool = True):
        _check(load_library().vlb_timing_enable(self._h, 1 if on else 0), "vlb_timing_enable")

    def timing_query(self):
        """List of dicts per stage-kernel instantiation: bits (64 FP64, 32 FP32), launches,
        total_ms, alg_bytes."""
        G = 64
        ng = ctypes.c_int()
        bits = (ctypes.c_int * G)()
        launches = (ctypes.c_long * G)()
        ms, by = np.zeros(G), np.zeros(G)
        _check(load_library().vlb_timing_query(self._h, G, ctypes.byref(ng), bits, launches, _ptr(ms), _ptr(by)),
               "vlb_timing_query")
        return [dict(bits=bits[i], launches=launches[i], total_ms=ms[i], alg_bytes=by[i]) for i in range(ng.value)]

    def velocities(self, b: int):
        i = self.info[b]
        p1, w1, p2, w2 = np.empty(i["nodes1"]), np.empty(i["nodes1"]), np.empty(i["nodes2"]), np.empty(i["nodes2"])
        _check(load_library().vlb_batch_velocities(self._h, b, _ptr(p1), _ptr(w1), _ptr(p2), _ptr(w2)),
               "vlb_batch_velocities")
        return p1, w1, p2, w2

    # ------------------------------------------------------------------ warm start
    @property
    def ncells(self) -> int:
        return sum(i["N_R"] for i in self.info)

    def surrogate_samples(self):
        """(X, T) float32 arrays [cells][4]: surrogate inputs and targets of the current state."""
        X = np.empty((self.ncells, 4), dtype=np.float32)
        T = np.empty((self.ncells, 4), dtype=np.float32)
        _check(load_library().vlb_batch_surrogate_samples(self._h, _fptr(X), _fptr(T), self.ncells),
               "vlb_batch_surrogate_samples")
        return X, T

    def warm_start(self, mlp: "Mlp", probe_steps: int = 1000) -> np.ndarray:
        """Initial states from the surrogate (cold start where the acceptance probe rejects it);
        returns the per-instance 0/1 array of warm starts kept."""
        used = (ctypes.c_int * self.B)()
        _check(load_library().vlb_batch_warm_start(self._h, mlp._h, probe_steps, used), "vlb_batch_warm_start")
        return np.array(list(used), dtype=np.int32)

    def set_stall_window(self, steps: int):
        """Steps without a new residual low after which run_to_steady restarts a warm-started
        instance from the cold rest state."""
        _check(load_library().vlb_batch_set_stall_window(self._h, steps), "vlb_batch_set_stall_window")

    def warm_report(self):
        """(on_warm, fallback_at) per instance: 1 while still on the warm start; the step of a
        cold restart (-1 none)."""
        on = (ctypes.c_int * self.B)()
        at = (ctypes.c_long * self.B)()
        _check(load_library().vlb_batch_warm_report(self._h, on, at), "vlb_batch_warm_report")
        return np.array(list(on), dtype=np.int32), np.array(list(at), dtype=np.int64)


def couette_step_noalloc(descs, F, nsteps: int, stream=None) -> np.ndarray:
    """nsteps FP64 RK3 steps of the instances `descs` on the device state F (a contiguous
    float64 torch tensor in the layout of Batch.get_state, updated in place) through the
    library's no-allocation entry point; returns the residual of the last step per instance."""
    import torch
    if not (isinstance(F, torch.Tensor) and F.is_cuda and F.dtype == torch.float64 and F.is_contiguous()):
        raise TypeError("F must be a contiguous float64 CUDA tensor")
    descs = list(descs)
    arr = (_CouetteDesc * len(descs))(*[d._c() for d in descs])
    st = stream if stream is not None else torch.cuda.current_stream(F.device)
    r = np.empty(len(descs))
    _check(load_library().vlb_couette_step_noalloc(len(descs), arr, ctypes.c_void_p(F.data_ptr()), nsteps, _ptr(r),
                                                   ctypes.c_void_p(st.cuda_stream)), "vlb_couette_step_noalloc")
    return r


def _fptr(a: np.ndarray):
    assert a.dtype == np.float32 and a.flags.c_contiguous
    return a.ctypes.data_as(_fp)


def mlp_param_count(width: int = 128, depth: int = 3) -> int:
    n = ctypes.c_size_t()
    _check(load_library().vlb_mlp_param_count(width, depth, ctypes.byref(n)), "vlb_mlp_param_count")
    return n.value


class Mlp:
    """The warm-start surrogate network on the GPU (parameters, Adam state, buffers in
    library-owned device memory; work on torch's current stream)."""

    def __init__(self, params: np.ndarray, width: int = 128, depth: int = 3, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the surrogate runs on the GPU only")
        self._torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.width, self.depth = width, depth
        self.n_params = mlp_param_count(width, depth)
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        if p.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {p.size}")
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(load_library().vlb_mlp_create(ctypes.byref(h), width, depth, _fptr(p),
                                             ctypes.c_void_p(self.stream.cuda_stream)), "vlb_mlp_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load_library().vlb_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        _check(load_library().vlb_mlp_get_params(self._h, _fptr(out), out.size), "vlb_mlp_get_params")
        return out

    def set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        _check(load_library().vlb_mlp_set_params(self._h, _fptr(p), p.size), "vlb_mlp_set_params")

    def _dev(self, a):
        """float32 [n][4] device tensor of a (host array or device tensor)."""
        t = self._torch
        if isinstance(a, t.Tensor):
            a = a.to(device=self.device, dtype=t.float32).contiguous()
        else:
            a = t.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(self.device)
        if a.dim() != 2 or a.shape[1] != 4:
            raise ValueError("expected an [n][4] array")
        return a

    def forward(self, X, bf16: bool = False) -> np.ndarray:
        Xd = self._dev(X)
        Y = self._torch.empty_like(Xd)
        _check(load_library().vlb_mlp_forward(self._h, ctypes.c_void_p(Xd.data_ptr()), Xd.shape[0],
                                              ctypes.c_void_p(Y.data_ptr()), 1 if bf16 else 0), "vlb_mlp_forward")
        self.stream.synchronize()
        return Y.cpu().numpy()

    def loss_grad(self, X, T):
        Xd, Td = self._dev(X), self._dev(T)
        loss = ctypes.c_float()
        g = np.empty(self.n_params, dtype=np.float32)
        _check(load_library().vlb_mlp_loss_grad(self._h, ctypes.c_void_p(Xd.data_ptr()), ctypes.c_void_p(Td.data_ptr()),
                                                Xd.shape[0], ctypes.byref(loss), _fptr(g)), "vlb_mlp_loss_grad")
        return loss.value, g

    def adam_step(self, grad=None, lr: float = 1e-3):
        gp = _fptr(np.ascontiguousarray(grad, dtype=np.float32)) if grad is not None else None
        _check(load_library().vlb_mlp_adam_step(self._h, gp, lr), "vlb_mlp_adam_step")

    def train(self, X, T, order: np.ndarray, batch: int = 512, lr: float = 1e-3) -> float:
        """Adam over the mini-batches of rows `order` of the samples (X, T): one call per
        epoch with a fresh permutation.  Returns the mean mini-batch loss."""
        Xd, Td = self._dev(X), self._dev(T)
        o = np.ascontiguousarray(order, dtype=np.int32)
        loss = ctypes.c_float()
        _check(load_library().vlb_mlp_train(self._h, ctypes.c_void_p(Xd.data_ptr()), ctypes.c_void_p(Td.data_ptr()),
                                            Xd.shape[0], o.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), o.size,
                                            batch, lr, ctypes.byref(loss)), "vlb_mlp_train")
        return loss.value


class Channel:
    """B expanding channels advanced together on one GPU, in FP64 or (VLB_MIXED) with
    FP32 stage kernels on weight-scaled populations."""

    def __init__(self, descs, precision: int = VLB_FP64, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the vielbein LB library runs on the GPU only")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.descs = list(descs)
        self.B = len(self.descs)
        arr = (_ChannelDesc * self.B)(*[d._c() for d in self.descs])
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        self.precision = precision
        lib = load_library()
        # device memory from torch's allocator, bound as the batch's workspace
        _check(lib.vlb_channel_create_deferred(ctypes.byref(h), self.B, arr, precision,
                                               ctypes.c_void_p(self.stream.cuda_stream)), "vlb_channel_create_deferred")
        self._h = h
        nbytes = ctypes.c_size_t()
        _check(lib.vlb_channel_workspace_bytes(h, ctypes.byref(nbytes)), "vlb_channel_workspace_bytes")
        self._ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        aligned = (self._ws.data_ptr() + 255) & ~255
        _check(lib.vlb_channel_bind_workspace(h, ctypes.c_void_p(aligned), nbytes.value), "vlb_channel_bind_workspace")
        n = ctypes.c_size_t()
        _check(load_library().vlb_channel_state_size(h, ctypes.byref(n)), "vlb_channel_state_size")
        self.state_size = n.value
        self.info = []
        for b in range(self.B):
            NL, NX, NV = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            dt, off = ctypes.c_double(), ctypes.c_size_t()
            _check(load_library().vlb_channel_info(h, b, ctypes.byref(NL), ctypes.byref(NX), ctypes.byref(NV),
                                                   ctypes.byref(dt), ctypes.byref(off)), "vlb_channel_info")
            self.info.append(dict(N_lambda=NL.value, N_xi=NX.value, NV=NV.value, dt=dt.value, offset=off.value))

    def close(self):
        if getattr(self, "_h", None):
            load_library().vlb_channel_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def instance_view(self, state, b):
        i = self.info[b]
        n = 2 * i["N_xi"] * i["N_lambda"] * i["NV"]
        return state[i["offset"]:i["offset"] + n].reshape(2, i["N_xi"], i["N_lambda"], i["NV"])

    def get_state(self):
        out = np.empty(self.state_size)
        _check(load_library().vlb_channel_get_state(self._h, _ptr(out), out.size), "vlb_channel_get_state")
        return out

    def set_state(self, state):
        s = np.ascontiguousarray(state, dtype=np.float64).ravel()
        _check(load_library().vlb_channel_set_state(self._h, _ptr(s), s.size), "vlb_channel_set_state")

    def get_instance_state(self, b: int) -> np.ndarray:
        i = self.info[b]
        out = np.empty((2, i["N_xi"], i["N_lambda"], i["NV"]))
        _check(load_library().vlb_channel_get_instance_state(self._h, b, _ptr(out), out.size),
               "vlb_channel_get_instance_state")
        return out

    def set_instance_state(self, b: int, F):
        s = np.ascontiguousarray(F, dtype=np.float64).ravel()
        _check(load_library().vlb_channel_set_instance_state(self._h, b, _ptr(s), s.size),
               "vlb_channel_set_instance_state")

    def init_equilibrium(self, b: int, n, u1, u2, T):
        """Instance b set to the local equilibrium of per-cell fields ([N_xi][N_lambda] each)."""
        i = self.info[b]
        shp = (i["N_xi"], i["N_lambda"])
        a = [np.ascontiguousarray(np.broadcast_to(np.asarray(x, dtype=np.float64), shp)) for x in (n, u1, u2, T)]
        _check(load_library().vlb_channel_init_equilibrium(self._h, b, *[_ptr(x) for x in a]),
               "vlb_channel_init_equilibrium")

    def set_open_bc(self, b: int, end: int, n: float, T: float):
        """Reservoir at end 0 (inlet) or 1 (outlet) of instance b: rest Maxwellian (n, T)."""
        _check(load_library().vlb_channel_set_open_bc(self._h, b, end, n, T), "vlb_channel_set_open_bc")

    def total_mass(self) -> np.ndarray:
        out = np.empty(self.B)
        _check(load_library().vlb_channel_total_mass(self._h, _ptr(out)), "vlb_channel_total_mass")
        return out

    def last_run_seconds(self) -> float:
        s = ctypes.c_double()
        _check(load_library().vlb_channel_last_run_seconds(self._h, ctypes.byref(s)), "vlb_channel_last_run_seconds")
        return s.value

    def step(self, nsteps: int = 1):
        _check(load_library().vlb_channel_step(self._h, nsteps), "vlb_channel_step")

    def step_fp64(self, nsteps: int = 1):
        _check(load_library().vlb_channel_step_fp64(self._h, nsteps), "vlb_channel_step_fp64")

    def fp32_steps(self) -> int:
        n = ctypes.c_long()
        _check(load_library().vlb_channel_fp32_steps(self._h, ctypes.byref(n)), "vlb_channel_fp32_steps")
        return n.value

    def apply_L(self):
        out = np.empty(self.state_size)
        _check(load_library().vlb_channel_apply_L(self._h, _ptr(out), out.size), "vlb_channel_apply_L")
        return out

    def residual(self):
        r = np.empty(self.B)
        _check(load_library().vlb_channel_residual(self._h, _ptr(r)), "vlb_channel_residual")
        return r

    def moments(self, b: int):
        i = self.info[b]
        shp = (i["N_xi"], i["N_lambda"])
        outs = [np.empty(shp) for _ in range(5)]
        _check(load_library().vlb_channel_moments(self._h, b, *[_ptr(o) for o in outs]), "vlb_channel_moments")
        return dict(zip(("n", "u1", "u2", "T", "content"), outs))

    def set_graphs(self, enable: bool):
        _check(load_library().vlb_channel_set_graphs(self._h, int(bool(enable))), "vlb_channel_set_graphs")

    def flow_fields(self, b: int) -> dict:
        """Cartesian velocity ux, uy, pressure P, vorticity omega ([N_xi][N_lambda]), stream
        function psi ([N_xi][N_lambda + 1]) and wall pressures Pw ([2][N_xi]) of instance b."""
        i = self.info[b]
        NX, NL = i["N_xi"], i["N_lambda"]
        names = ("ux", "uy", "P", "psi", "omega", "Pw")
        outs = {k: np.empty((NX, NL)) for k in ("ux", "uy", "P", "omega")}
        outs["psi"] = np.empty((NX, NL + 1))
        outs["Pw"] = np.empty((2, NX))
        _check(load_library().vlb_channel_flow_fields(self._h, b, *[_ptr(outs[k]) for k in names]),
               "vlb_channel_flow_fields")
        return outs

    def run_to_steady(self, tol: float, max_steps: int, check_every: int = 100):
        steps = (ctypes.c_long * self.B)()
        r = np.empty(self.B)
        st = load_library().vlb_channel_run_to_steady(self._h, tol, max_steps, check_every, steps, _ptr(r))
        if st not in (0, -5):
            _check(st, "vlb_channel_run_to_steady")
        return np.array(list(steps)), r, st == 0
