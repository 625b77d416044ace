"""Python binding of the gfx950 delay-and-sum library (``include/das.h``).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libdas_mi355x.so``.  PyTorch provides device memory and the
current HIP stream.  If the library is missing, every call raises: there is
no CPU or PyTorch fallback.

The functions carry the C names (``das_plan_create``, ``das_prepare``,
``das_forward``, ``das_adjoint``, ``das_grad_sound_speed``, ...); ``Plan``
wraps them for convenience and ``DASFunction`` makes the forward pass
differentiable with respect to channel data and sound speed.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdas_mi355x.so")

DAS_OK, DAS_ERR_INVALID_ARG, DAS_ERR_UNSUPPORTED, DAS_ERR_HIP, DAS_ERR_OOM = 0, -1, -2, -3, -4
TX_NONE, TX_PLANE, TX_DIVERGING = 0, 1, 2
STORE = {"f32": 0, "f16": 1, "bf16": 2, "fp8": 3}
APOD_UNIFORM, APOD_HANN = 0, 1
ALGO = {"auto": 0, "plain": 1, "tiled": 2, "mfma": 3}
ALGO_NAME = {v: k for k, v in ALGO.items()}
DAS_INTERP_LINEAR, DAS_INTERP_CUBIC = 0, 1
MFMA_FORM = {"auto": 0, "column": 1, "slab": 2, "persistent": 3, "column_fp8": 4, "slab_fp8": 5}


class DasError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


class DasTx(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("vec", ctypes.c_double * 3),
                ("path_offset", ctypes.c_double)]


class DasGrid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("spacing", ctypes.c_double * 3),
                ("dims", ctypes.c_int32 * 3)]


class DasConfig(ctypes.Structure):
    _fields_ = [
        ("num_elements", ctypes.c_int32),
        ("element_pos", ctypes.POINTER(ctypes.c_double)),
        ("element_normal", ctypes.POINTER(ctypes.c_double)),
        ("num_tx", ctypes.c_int32),
        ("tx", ctypes.POINTER(DasTx)),
        ("grid", DasGrid),
        ("num_samples", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("sound_speed", ctypes.c_double),
        ("fs", ctypes.c_double),
        ("t0", ctypes.c_double),
        ("apod", ctypes.c_int32),
        ("f_number", ctypes.c_double),
        ("storage", ctypes.c_int32),
        ("algo", ctypes.c_int32),
    ]


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int32


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2606_13259_amd.build` "
                "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "das_plan_create": [ctypes.POINTER(_P), ctypes.POINTER(DasConfig), ctypes.c_int],
            "das_plan_destroy": [_P],
            "das_plan_set_sound_speed": [_P, ctypes.c_double],
            "das_plan_set_tx_weights": [_P, _P],
            "das_plan_set_algo": [_P, _I],
            "das_plan_get_algo": [_P, _I, ctypes.POINTER(_I)],
            "das_workspace_bytes": [_P, _I, ctypes.POINTER(ctypes.c_size_t)],
            "das_prepare": [_P, _P, _I, _I, _I, _P, _P],
            "das_forward": [_P, _P, _I, _P, _P],
            "das_adjoint": [_P, _P, _I, _P, _P],
            "das_grad_sound_speed": [_P, _P, _P, _I, _P, _P],
            "das_forward_batched": [_I, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_I),
                                    ctypes.POINTER(_P), _P],
            "das_autotune": [_P, _I, _P],
            "das_plan_get_tile": [_P, ctypes.POINTER(_I)],
            "das_plan_set_tile": [_P, _I],
            "das_tile_shape": [_I, ctypes.POINTER(_I)],
            "das_debug_delays": [_P, _I, _I, _I, _I, _I, _P, _P],
            "das_plan_set_iq": [_P, _I, ctypes.c_double],
            "das_plan_set_interp": [_P, _I],
            "das_plan_set_mfma_form": [_P, _I],
            "das_plan_get_mfma_form": [_P, ctypes.POINTER(_I)],
            "das_clutter_workspace_bytes": [_I, ctypes.POINTER(ctypes.c_size_t)],
            "das_clutter_filter": [_P, _I, ctypes.c_int64, _I, _I, _P, _P, _P, _P, _P],
            "das_clutter_filter_noalloc": [_P, _I, ctypes.c_int64, _I, _I, _P, _P, _P, _P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.das_num_tile_shapes.restype = ctypes.c_int32
        L.das_num_tile_shapes.argtypes = []
        for name in ("das_status_string", "das_last_error", "das_version"):
            getattr(L, name).restype = ctypes.c_char_p
        L.das_status_string.argtypes = [ctypes.c_int]
        L.das_last_error.argtypes = []
        L.das_version.argtypes = []
        _lib = L
    return _lib


def _check(st: int, where: str):
    if st != DAS_OK:
        raise DasError(st, where, lib().das_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def make_config(geom, max_batch: int = 1, storage: str = "f32", algo: str = "auto"):
    """A DasConfig (plus the host arrays it points to) from a geometry object
    with the attributes of ``synth.Geometry``."""
    pos = np.ascontiguousarray(np.asarray(geom.elem_pos, np.float64).reshape(-1, 3))
    nrm = getattr(geom, "elem_normal", None)
    nrm = None if nrm is None else np.ascontiguousarray(np.asarray(nrm, np.float64).reshape(-1, 3))
    kinds = np.asarray(geom.tx_kind)
    Q = kinds.shape[0]
    txs = (DasTx * Q)()
    for q in range(Q):
        txs[q].kind = int(kinds[q])
        for i in range(3):
            txs[q].vec[i] = float(np.asarray(geom.tx_vec, np.float64).reshape(Q, 3)[q, i])
        txs[q].path_offset = float(np.asarray(geom.tx_offset, np.float64)[q])
    cfg = DasConfig()
    cfg.num_elements = pos.shape[0]
    cfg.element_pos = pos.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    cfg.element_normal = (None if nrm is None else nrm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    cfg.num_tx = Q
    cfg.tx = ctypes.cast(txs, ctypes.POINTER(DasTx))
    for i in range(3):
        cfg.grid.origin[i] = float(geom.grid_origin[i])
        cfg.grid.spacing[i] = float(geom.grid_spacing[i])
        cfg.grid.dims[i] = int(geom.grid_dims[i])
    cfg.num_samples = int(geom.num_samples)
    cfg.max_batch = int(max_batch)
    cfg.sound_speed = float(geom.c)
    cfg.fs = float(geom.fs)
    cfg.t0 = float(geom.t0)
    cfg.apod = int(geom.apod)
    cfg.f_number = float(geom.f_number)
    cfg.storage = STORE[storage] if isinstance(storage, str) else int(storage)
    cfg.algo = ALGO[algo] if isinstance(algo, str) else int(algo)
    return cfg, (pos, nrm, txs)


# ---------------------------------------------------------------------------
# C entry points
# ---------------------------------------------------------------------------

def das_plan_create(cfg: DasConfig, device: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().das_plan_create(ctypes.byref(h), ctypes.byref(cfg), int(device)), "das_plan_create")
    return h


def das_plan_destroy(h):
    _check(lib().das_plan_destroy(h), "das_plan_destroy")


def das_workspace_bytes(h, batch: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().das_workspace_bytes(h, int(batch), ctypes.byref(out)), "das_workspace_bytes")
    return int(out.value)


def das_prepare(h, y: torch.Tensor, b0: int, nb: int, batch_total: int, ws: torch.Tensor):
    _check(lib().das_prepare(h, _ptr(y), int(b0), int(nb), int(batch_total), _ptr(ws),
                             _stream(y.device)), "das_prepare")


def das_forward(h, ws: torch.Tensor, batch: int, x: torch.Tensor):
    _check(lib().das_forward(h, _ptr(ws), int(batch), _ptr(x), _stream(x.device)), "das_forward")


def das_adjoint(h, gx: torch.Tensor, batch: int, gy: torch.Tensor):
    _check(lib().das_adjoint(h, _ptr(gx), int(batch), _ptr(gy), _stream(gy.device)), "das_adjoint")


def das_grad_sound_speed(h, y: torch.Tensor, gx: torch.Tensor, batch: int, out: torch.Tensor):
    _check(lib().das_grad_sound_speed(h, _ptr(y), _ptr(gx), int(batch), _ptr(out),
                                      _stream(out.device)), "das_grad_sound_speed")


def das_forward_batched(plans, ws_list, batches, xs):
    n = len(plans)
    hp = (_P * n)(*[p.value if isinstance(p, ctypes.c_void_p) else p for p in plans])
    wp = (_P * n)(*[w.data_ptr() for w in ws_list])
    bp = (_I * n)(*[int(b) for b in batches])
    xp = (_P * n)(*[x.data_ptr() for x in xs])
    _check(lib().das_forward_batched(n, hp, wp, bp, xp, _stream(xs[0].device)), "das_forward_batched")


def das_autotune(h, batch: int, device):
    _check(lib().das_autotune(h, int(batch), _stream(device)), "das_autotune")


def das_clutter_workspace_bytes(T: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().das_clutter_workspace_bytes(int(T), ctypes.byref(n)), "das_clutter_workspace_bytes")
    return n.value


def das_clutter_filter(x: torch.Tensor, k_lo: int, k_hi: int, sv: torch.Tensor, power: torch.Tensor,
                       xf: Optional[torch.Tensor], ws: torch.Tensor):
    T = x.shape[0]
    N = x.numel() // T
    _check(lib().das_clutter_filter(_ptr(x), int(T), int(N), int(k_lo), int(k_hi), _ptr(sv), _ptr(power),
                                    _ptr(xf), _ptr(ws), _stream(x.device)), "das_clutter_filter")


def das_clutter_filter_noalloc(x: torch.Tensor, k_lo: int, k_hi: int, sv: torch.Tensor,
                               power: torch.Tensor, xf: Optional[torch.Tensor]):
    T = x.shape[0]
    N = x.numel() // T
    _check(lib().das_clutter_filter_noalloc(_ptr(x), int(T), int(N), int(k_lo), int(k_hi), _ptr(sv),
                                            _ptr(power), _ptr(xf), _stream(x.device)),
           "das_clutter_filter_noalloc")


def clutter_filter(x: torch.Tensor, k_lo: int, k_hi: Optional[int] = None, filtered: bool = False):
    """Rank-truncation clutter filter of an ensemble x[T, ...] (float32, on a
    GPU): keeps singular components k_lo .. k_hi-1 of the Casorati matrix.
    Returns (singular values [T], power Doppler [...], filtered ensemble or
    None)."""
    assert x.dtype == torch.float32 and x.is_contiguous() and x.is_cuda
    T = x.shape[0]
    k_hi = T if k_hi is None else k_hi
    with torch.cuda.device(x.device):
        ws = torch.empty(das_clutter_workspace_bytes(T), dtype=torch.uint8, device=x.device)
        sv = torch.empty(T, dtype=torch.float32, device=x.device)
        pw = torch.empty(x.shape[1:], dtype=torch.float32, device=x.device)
        xf = torch.empty_like(x) if filtered else None
        das_clutter_filter(x, k_lo, k_hi, sv, pw, xf, ws)
    return sv, pw, xf


def das_debug_delays(h, q, m0, m1, n0, n1, out: torch.Tensor):
    _check(lib().das_debug_delays(h, int(q), int(m0), int(m1), int(n0), int(n1), _ptr(out),
                                  _stream(out.device)), "das_debug_delays")


def das_tile_shape(idx: int):
    dims = (_I * 3)()
    _check(lib().das_tile_shape(int(idx), dims), "das_tile_shape")
    return tuple(int(v) for v in dims)


def das_num_tile_shapes() -> int:
    return int(lib().das_num_tile_shapes())


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------

class Plan:
    """Owns a das_plan for one geometry on one device."""

    def __init__(self, geom, max_batch: int = 1, storage: str = "f32", algo: str = "auto",
                 device: int = 0):
        self.geom = geom
        self.device = torch.device("cuda", device)
        self.max_batch = int(max_batch)
        self.storage = storage
        cfg, self._keep = make_config(geom, max_batch, storage, algo)
        self.handle = das_plan_create(cfg, device)
        self.Q, self.M, self.K = int(cfg.num_tx), int(cfg.num_elements), int(cfg.num_samples)
        self.N = int(np.prod(geom.grid_dims))
        self._w_tx = None
        self.c = float(geom.c)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            das_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- settings
    def set_sound_speed(self, c: float):
        _check(lib().das_plan_set_sound_speed(self.handle, float(c)), "das_plan_set_sound_speed")
        self.c = float(c)

    def set_tx_weights(self, w_tx: Optional[torch.Tensor]):
        if w_tx is not None:
            assert w_tx.dtype == torch.float32 and w_tx.is_contiguous() and w_tx.numel() == self.Q * self.N
        self._w_tx = w_tx
        _check(lib().das_plan_set_tx_weights(self.handle, _ptr(w_tx)), "das_plan_set_tx_weights")

    def set_iq(self, fc: float, enable: bool = True):
        """Complex baseband mode: batch items are (I, Q) pairs demodulated at
        fc (Hz); the forward remodulates every term by exp(i 2 pi fc tau) and
        the adjoint applies the conjugate phase."""
        _check(lib().das_plan_set_iq(self.handle, int(bool(enable)), float(fc)), "das_plan_set_iq")

    def set_interp(self, interp: str):
        """Sample interpolation: "linear" (Eq. (2)) or "cubic" (four-point
        Lagrange through samples k-1 .. k+2; windowed algorithm, f32 storage)."""
        code = {"linear": DAS_INTERP_LINEAR, "cubic": DAS_INTERP_CUBIC}[interp]
        _check(lib().das_plan_set_interp(self.handle, code), "das_plan_set_interp")

    def set_mfma_form(self, form: str):
        """Launch form of the MFMA algorithm: "auto", "column" (4x4x4 voxel
        columns per wavefront), "slab" (8x8x1 slabs), "persistent", or for FP8
        storage "column_fp8" / "slab_fp8" (FP8 matrix operands)."""
        _check(lib().das_plan_set_mfma_form(self.handle, MFMA_FORM[form]), "das_plan_set_mfma_form")

    def mfma_form(self) -> str:
        v = _I()
        _check(lib().das_plan_get_mfma_form(self.handle, ctypes.byref(v)), "das_plan_get_mfma_form")
        return {k: f for f, k in MFMA_FORM.items()}[v.value]

    def set_algo(self, algo: str):
        _check(lib().das_plan_set_algo(self.handle, ALGO[algo]), "das_plan_set_algo")

    def algo(self, batch: int = 1) -> str:
        a = _I()
        _check(lib().das_plan_get_algo(self.handle, int(batch), ctypes.byref(a)), "das_plan_get_algo")
        return ALGO_NAME[a.value]

    def tile(self) -> int:
        t = _I()
        _check(lib().das_plan_get_tile(self.handle, ctypes.byref(t)), "das_plan_get_tile")
        return t.value

    def set_tile(self, idx: int):
        _check(lib().das_plan_set_tile(self.handle, int(idx)), "das_plan_set_tile")

    def autotune(self, batch: int = 1) -> int:
        das_autotune(self.handle, batch, self.device)
        return self.tile()

    # -- compute
    def workspace(self, batch: int) -> torch.Tensor:
        return torch.empty(das_workspace_bytes(self.handle, batch), dtype=torch.uint8,
                           device=self.device)

    def prepare(self, y: torch.Tensor, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
        """y: [B, Q, M, K] float32 on the plan's device -> prepared workspace."""
        y = _as_batched(y, self)
        B = y.shape[0]
        ws = self.workspace(B) if ws is None else ws
        das_prepare(self.handle, y, 0, B, B, ws)
        return ws

    def forward_ws(self, ws: torch.Tensor, batch: int, x: Optional[torch.Tensor] = None):
        x = torch.empty(batch, self.N, dtype=torch.float32, device=self.device) if x is None else x
        das_forward(self.handle, ws, batch, x)
        return x

    def forward(self, y: torch.Tensor) -> torch.Tensor:
        """x[B, N] = DAS(y[B, Q, M, K])."""
        y = _as_batched(y, self)
        return self.forward_ws(self.prepare(y), y.shape[0])

    def adjoint(self, gx: torch.Tensor) -> torch.Tensor:
        gx = gx.reshape(-1, self.N).contiguous()
        assert gx.dtype == torch.float32 and gx.device == self.device
        B = gx.shape[0]
        gy = torch.empty(B, self.Q, self.M, self.K, dtype=torch.float32, device=self.device)
        das_adjoint(self.handle, gx, B, gy)
        return gy

    def grad_sound_speed(self, y: torch.Tensor, gx: torch.Tensor) -> torch.Tensor:
        y = _as_batched(y, self)
        gx = gx.reshape(-1, self.N).contiguous()
        out = torch.empty(1, dtype=torch.float32, device=self.device)
        das_grad_sound_speed(self.handle, y, gx, y.shape[0], out)
        return out[0]

    def debug_delays(self, q: int, m0: int, m1: int, n0: int, n1: int) -> torch.Tensor:
        out = torch.empty(m1 - m0, n1 - n0, dtype=torch.float64, device=self.device)
        das_debug_delays(self.handle, q, m0, m1, n0, n1, out)
        return out


def _as_batched(y: torch.Tensor, plan: Plan) -> torch.Tensor:
    if y.dim() == 3:
        y = y.unsqueeze(0)
    if y.dtype != torch.float32 or not y.is_contiguous() or y.device != plan.device:
        raise ValueError("channel data must be a contiguous float32 tensor [B, Q, M, K] on "
                         f"{plan.device}")
    if tuple(y.shape[1:]) != (plan.Q, plan.M, plan.K):
        raise ValueError(f"channel data shape {tuple(y.shape)} does not match the plan "
                         f"(Q, M, K) = {(plan.Q, plan.M, plan.K)}")
    return y


class DASFunction(torch.autograd.Function):
    """x = DAS_c(y), differentiable in y (through the adjoint kernel) and in
    the sound speed c (through the gradient kernel).  Only (y, c) are saved;
    nothing of the forward volume or the delays is stored."""

    @staticmethod
    def forward(ctx, y, c, plan: Plan):
        plan.set_sound_speed(float(c))
        ctx.plan = plan
        ctx.save_for_backward(y, c)
        return plan.forward(y.detach().contiguous())

    @staticmethod
    def backward(ctx, gx):
        y, c = ctx.saved_tensors
        plan = ctx.plan
        plan.set_sound_speed(float(c))
        gx = gx.contiguous()
        gy = plan.adjoint(gx).reshape(y.shape) if ctx.needs_input_grad[0] else None
        gc = None
        if ctx.needs_input_grad[1]:
            gc = plan.grad_sound_speed(y.detach().contiguous(), gx).to(c.dtype).reshape(c.shape)
        return gy, gc, None
