"""Python binding of libqla (C ABI in include/qla.h).

The functions here carry the C names and only marshal arguments: every
step of the method runs in the HIP kernels of ``libqla.so``. PyTorch
provides device memory and streams. If the library has not been built
the import fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqla.so")

QLA_OK, QLA_EINVAL, QLA_ENOMEM, QLA_EDEVICE, QLA_ESTATE = 0, -1, -2, -3, -4
POT_MODES = {"eq23": 0, "eq28": 1}
BETA_SCALES = {"phys": 0, "lattice": 1, "off": 2}
POLARISATIONS = {"both": 0, "tm": 1, "te": 2}
V_FORMS = {"printed": 0, "skew": 1}
_STATUS = {0: "QLA_OK", -1: "QLA_EINVAL", -2: "QLA_ENOMEM", -3: "QLA_EDEVICE", -4: "QLA_ESTATE"}


class QlaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("delta", ctypes.c_double),
                ("pot_mode", ctypes.c_int32), ("beta_scale", ctypes.c_int32),
                ("polarisation", ctypes.c_int32), ("v_form", ctypes.c_int32)]


class Diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("energy", ctypes.c_double),
                ("divB_max", ctypes.c_double), ("divB_l2", ctypes.c_double),
                ("B_max", ctypes.c_double), ("B_l2", ctypes.c_double),
                ("divD_max", ctypes.c_double), ("divD_l2", ctypes.c_double),
                ("D_max", ctypes.c_double)]

    def as_dict(self) -> Dict[str, float]:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Launch(ctypes.Structure):
    _fields_ = [("seg_rows", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("graph_steps", ctypes.c_int32), ("steps_per_pass", ctypes.c_int32),
                ("stream_loads", ctypes.c_int32), ("vacuum_rows", ctypes.c_int32)]

    def as_dict(self) -> Dict[str, int]:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class Instance(ctypes.Structure):
    _fields_ = [("p", Params), ("d_n", ctypes.c_void_p), ("d_q", ctypes.c_void_p),
                ("d_q_pong", ctypes.c_void_p)]


_lib = None

# name -> (argtypes, restype); the exported surface of include/qla.h
_SIGNATURES = {
    "qla_workspace_size": ([ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "qla_batch_workspace_size": ([ctypes.c_int32, ctypes.POINTER(Instance),
                                  ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "qla_init": ([ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "qla_init_batch": ([ctypes.c_int32, ctypes.POINTER(Instance), ctypes.c_void_p, ctypes.c_void_p,
                        ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "qla_count": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "qla_step": ([ctypes.c_void_p, ctypes.c_int64], ctypes.c_int),
    "qla_energy": ([ctypes.c_void_p, ctypes.POINTER(Diag)], ctypes.c_int),
    "qla_energy_noalloc": ([ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                            ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "qla_fields": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    "qla_fields_at": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32],
                      ctypes.c_int),
    "qla_load_at": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32], ctypes.c_int),
    "qla_get_launch": ([ctypes.c_void_p, ctypes.POINTER(Launch)], ctypes.c_int),
    "qla_set_launch": ([ctypes.c_void_p, ctypes.POINTER(Launch)], ctypes.c_int),
    "qla_state": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "qla_state_at": ([ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "qla_free": ([ctypes.c_void_p], None),
    "qla_last_error": ([], ctypes.c_char_p),
}


def lib() -> ctypes.CDLL:
    """The loaded libqla.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python -m paper_2301_13601_amd.build")
        # torch first: its HIP runtime is then the one libqla.so binds to
        # (a second copy of the runtime, loaded ahead of torch's, does not
        # see the device torch has opened)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (argtypes, restype) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = argtypes
            fn.restype = restype
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != QLA_OK:
        raise QlaError(status, qla_last_error())


def make_params(nx: int, ny: int, delta: float, pot_mode: str = "eq28", beta_scale: str = "phys",
                polarisation: str = "both", v_form: str = "printed") -> Params:
    return Params(int(nx), int(ny), float(delta), POT_MODES[pot_mode], BETA_SCALES[beta_scale],
                  POLARISATIONS[polarisation], V_FORMS[v_form])


# ---------------------------------------------------------------------------
# The C entry points, one to one.
# ---------------------------------------------------------------------------

def qla_last_error() -> str:
    msg = lib().qla_last_error()
    return msg.decode() if msg else ""


def qla_workspace_size(params: Params) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().qla_workspace_size(ctypes.byref(params), ctypes.byref(out)))
    return int(out.value)


def qla_batch_workspace_size(instances) -> int:
    arr = (Instance * len(instances))(*instances)
    out = ctypes.c_size_t(0)
    _check(lib().qla_batch_workspace_size(len(instances), arr, ctypes.byref(out)))
    return int(out.value)


def qla_init_batch(instances, d_work: int, stream: int) -> ctypes.c_void_p:
    arr = (Instance * len(instances))(*instances)
    ctx = ctypes.c_void_p()
    _check(lib().qla_init_batch(len(instances), arr, ctypes.c_void_p(d_work), ctypes.c_void_p(stream),
                                ctypes.byref(ctx)))
    return ctx


def qla_count(ctx) -> int:
    out = ctypes.c_int32(0)
    _check(lib().qla_count(ctx, ctypes.byref(out)))
    return int(out.value)


def qla_init(params: Params, d_n: int, d_q: int, d_q_pong: int, d_work: int,
             stream: int) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(lib().qla_init(ctypes.byref(params), ctypes.c_void_p(d_n), ctypes.c_void_p(d_q),
                          ctypes.c_void_p(d_q_pong), ctypes.c_void_p(d_work),
                          ctypes.c_void_p(stream), ctypes.byref(ctx)))
    return ctx


def qla_step(ctx, nsteps: int) -> None:
    _check(lib().qla_step(ctx, int(nsteps)))


def qla_energy(ctx, count: int = 1):
    """One diagnostics dict per lattice (a single dict when count == 1)."""
    d = (Diag * count)()
    _check(lib().qla_energy(ctx, d))
    out = [x.as_dict() for x in d]
    return out[0] if count == 1 else out


def qla_energy_noalloc(params: Params, d_n: int, d_q: int, step: int, d_out: int, stream: int) -> None:
    """Enqueue the diagnostics of the state at d_q into the qla_diag at
    device address d_out (no allocation, no synchronisation)."""
    _check(lib().qla_energy_noalloc(ctypes.byref(params), ctypes.c_void_p(d_n), ctypes.c_void_p(d_q),
                                    int(step), ctypes.c_void_p(d_out), ctypes.c_void_p(stream)))


def qla_fields(ctx, dst: int, what: int, dst_is_host: bool) -> None:
    _check(lib().qla_fields(ctx, ctypes.c_void_p(dst), int(what), int(bool(dst_is_host))))


def qla_fields_at(ctx, index: int, dst: int, what: int, dst_is_host: bool) -> None:
    _check(lib().qla_fields_at(ctx, int(index), ctypes.c_void_p(dst), int(what), int(bool(dst_is_host))))


def qla_load_at(ctx, index: int, src: int, src_is_host: bool) -> None:
    _check(lib().qla_load_at(ctx, int(index), ctypes.c_void_p(src), int(bool(src_is_host))))


def qla_get_launch(ctx) -> Dict[str, int]:
    out = Launch()
    _check(lib().qla_get_launch(ctx, ctypes.byref(out)))
    return out.as_dict()


def qla_set_launch(ctx, seg_rows: int = 0, waves_per_block: int = 0, graph_steps: int = 0,
                   steps_per_pass: int = 0, stream_loads: int = 0, vacuum_rows: int = 0) -> None:
    req = Launch(int(seg_rows), int(waves_per_block), int(graph_steps), int(steps_per_pass), int(stream_loads),
                 int(vacuum_rows))
    _check(lib().qla_set_launch(ctx, ctypes.byref(req)))


def qla_state(ctx) -> int:
    p = ctypes.c_void_p()
    _check(lib().qla_state(ctx, ctypes.byref(p)))
    return int(p.value)


def qla_state_at(ctx, index: int) -> int:
    p = ctypes.c_void_p()
    _check(lib().qla_state_at(ctx, int(index), ctypes.byref(p)))
    return int(p.value)


def qla_free(ctx) -> None:
    lib().qla_free(ctx)


# ---------------------------------------------------------------------------
# Convenience owner of the device buffers (torch) around one context.
# ---------------------------------------------------------------------------

class Simulation:
    """One lattice on one GPU: n, two state buffers and the workspace as torch
    tensors, and the libqla context bound to them."""

    def __init__(self, n, q0, delta: float, pot_mode: str = "eq28", beta_scale: str = "phys",
                 device: str = "cuda:0", stream=None, polarisation: str = "both", v_form: str = "printed"):
        import torch

        self._torch = torch
        n_t = torch.as_tensor(np.ascontiguousarray(n, dtype=np.float32)) if isinstance(n, np.ndarray) else n
        q_t = torch.as_tensor(np.ascontiguousarray(q0, dtype=np.float32)) if isinstance(q0, np.ndarray) else q0
        if n_t.dim() != 3 or n_t.shape[0] != 3 or tuple(q_t.shape) != (6,) + tuple(n_t.shape[1:]):
            raise ValueError("expected n of shape (3, ny, nx) and q0 of shape (6, ny, nx)")
        self.ny, self.nx = int(n_t.shape[1]), int(n_t.shape[2])
        self.device = torch.device(device)
        self.n = n_t.to(self.device, torch.float32).contiguous()
        self.q = q_t.to(self.device, torch.float32).contiguous().clone()
        self.q_pong = torch.empty_like(self.q)
        self.params = make_params(self.nx, self.ny, delta, pot_mode, beta_scale, polarisation, v_form)
        nbytes = qla_workspace_size(self.params)
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = qla_init(self.params, self.n.data_ptr(), self.q.data_ptr(), self.q_pong.data_ptr(),
                            self.work.data_ptr(), self.stream.cuda_stream)

    def step(self, nsteps: int) -> None:
        qla_step(self.ctx, nsteps)

    def diagnostics(self) -> Dict[str, float]:
        return qla_energy(self.ctx)

    def fields(self, what: str = "Q") -> np.ndarray:
        out = np.empty((6, self.ny, self.nx), dtype=np.float32)
        qla_fields(self.ctx, out.ctypes.data, {"Q": 0, "EB": 1}[what], True)
        return out

    def launch(self) -> Dict[str, int]:
        return qla_get_launch(self.ctx)

    def set_launch(self, seg_rows: int = 0, waves_per_block: int = 0, graph_steps: int = 0,
                   steps_per_pass: int = 0, stream_loads: int = 0, vacuum_rows: int = 0) -> None:
        qla_set_launch(self.ctx, seg_rows, waves_per_block, graph_steps, steps_per_pass, stream_loads,
                       vacuum_rows)

    def state_tensor(self):
        """The device tensor that holds the current state (no copy)."""
        ptr = qla_state(self.ctx)
        return self.q if ptr == self.q.data_ptr() else self.q_pong

    def close(self) -> None:
        if self.ctx is not None:
            qla_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many lattices of uneven sizes stepped together (one kernel launch per
    step for the whole batch): per-lattice n, state buffers (torch) and one
    shared workspace."""

    def __init__(self, ns, q0s, deltas, pot_mode: str = "eq28", beta_scale: str = "phys",
                 device: str = "cuda:0", stream=None, polarisation: str = "both", v_form: str = "printed"):
        import torch

        if not (len(ns) == len(q0s) == len(deltas)) or len(ns) == 0:
            raise ValueError("need one n, q0 and delta per lattice")
        self.device = torch.device(device)
        self.n, self.q, self.q_pong, self.shapes = [], [], [], []
        insts = []
        def dev_tensor(a):
            if isinstance(a, torch.Tensor):
                return a.to(self.device, torch.float32).contiguous()
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(self.device)

        for n, q0, d in zip(ns, q0s, deltas):
            n_t = dev_tensor(n)
            q_t = dev_tensor(q0).clone()
            if n_t.dim() != 3 or n_t.shape[0] != 3 or tuple(q_t.shape) != (6,) + tuple(n_t.shape[1:]):
                raise ValueError("expected n of shape (3, ny, nx) and q0 of shape (6, ny, nx)")
            ny, nx = int(n_t.shape[1]), int(n_t.shape[2])
            qp = torch.empty_like(q_t)
            self.n.append(n_t)
            self.q.append(q_t)
            self.q_pong.append(qp)
            self.shapes.append((ny, nx))
            insts.append(Instance(make_params(nx, ny, d, pot_mode, beta_scale, polarisation, v_form), n_t.data_ptr(),
                                  q_t.data_ptr(), qp.data_ptr()))
        nbytes = qla_batch_workspace_size(insts)
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = qla_init_batch(insts, self.work.data_ptr(), self.stream.cuda_stream)
        self.count = len(insts)

    @property
    def sites(self) -> int:
        return sum(ny * nx for ny, nx in self.shapes)

    def step(self, nsteps: int) -> None:
        qla_step(self.ctx, nsteps)

    def diagnostics(self):
        return qla_energy(self.ctx, self.count) if self.count > 1 else [qla_energy(self.ctx, 1)]

    def fields(self, what: str = "Q"):
        total = sum(6 * ny * nx for ny, nx in self.shapes)
        flat = np.empty(total, dtype=np.float32)
        qla_fields(self.ctx, flat.ctypes.data, {"Q": 0, "EB": 1}[what], True)
        out, o = [], 0
        for ny, nx in self.shapes:
            out.append(flat[o:o + 6 * ny * nx].reshape(6, ny, nx))
            o += 6 * ny * nx
        return out

    def launch(self) -> Dict[str, int]:
        return qla_get_launch(self.ctx)

    def set_launch(self, seg_rows: int = 0, waves_per_block: int = 0, graph_steps: int = 0,
                   steps_per_pass: int = 0, stream_loads: int = 0, vacuum_rows: int = 0) -> None:
        qla_set_launch(self.ctx, seg_rows, waves_per_block, graph_steps, steps_per_pass, stream_loads,
                       vacuum_rows)

    def close(self) -> None:
        if self.ctx is not None:
            qla_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
