"""Learned warm start: binding of the t2s2_mlp_* and t2s2_tt_pack/unpack entries.

A systems addition around the method (the paper trains nothing): a network
maps an instance's parameters to TT cores that start the sweeps; the FP64
residual judges the start (t2s2_options.warm_judge) and the cold start stays
the fallback.  Argument marshalling only; every numerical step runs in
libt2s2's kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import numpy as np

from . import _lib
from ._lib import check, lib

def n_features(d: int) -> int:
    """beta (d), log10 eps, 4 amplitudes, 4 widths, 4 offsets: 20 for d = 7."""
    return d + 13


def features(params: Sequence[dict]) -> np.ndarray:
    """Network inputs of warm-start instances (n_features(d) each), scaled to
    about [-1, 1]: beta as is, log10(eps) + 3, amplitude - 1,
    (width - 0.35) / 0.15, 2 * offset."""
    rows = []
    for q in params:
        rows.append(np.concatenate([np.asarray(q["beta"], dtype=np.float64), [np.log10(q["eps"]) + 3.0],
                                    np.asarray(q["amp"]) - 1.0, (np.asarray(q["width"]) - 0.35) / 0.15,
                                    2.0 * np.asarray(q["offset"])]))
    return np.asarray(rows, dtype=np.float32)


def _torch():
    import torch
    return torch


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(t, cols: int, name: str, rows: Optional[int] = None):
    """The C ABI takes bare pointers: reject arrays of the wrong shape here."""
    torch = _torch()
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.dim() == 2 and t.shape[1] == cols
            and (rows is None or t.shape[0] == rows) and t.shape[0] >= 1):
        raise ValueError(f"{name} must be a contiguous float32 CUDA array of shape "
                         f"({rows if rows is not None else 'batch'}, {cols}), got {tuple(t.shape)} {t.dtype}")


def flat_size(n: Sequence[int], rank: int) -> int:
    d = len(n)
    ranks = [1] + [rank] * (d - 1) + [1]
    return int(sum(ranks[l] * n[l] * ranks[l + 1] for l in range(d)))


class Network:
    """t2s2_mlp: widths w_0 .. w_L, tanh hidden layers, linear output."""

    def __init__(self, widths: Sequence[int], seed: int = 0):
        self.widths = [int(w) for w in widths]
        h = C.c_void_p()
        arr = (C.c_int * len(self.widths))(*self.widths)
        check(lib().t2s2_mlp_create(len(self.widths) - 1, arr, C.c_ulonglong(seed), C.byref(h)))
        self._h = h
        cnt = C.c_longlong()
        check(lib().t2s2_mlp_param_count(self._h, C.byref(cnt)))
        self.param_count = int(cnt.value)

    def close(self):
        if getattr(self, "_h", None):
            lib().t2s2_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, which: int):
        torch = _torch()
        out = torch.empty(self.param_count, dtype=torch.float32, device="cuda")
        check(lib().t2s2_mlp_get_params(self._h, _ptr(out), which, _stream()))
        return out

    def params(self):
        return self._vec(0)

    def grad(self):
        return self._vec(1)

    def set_params(self, p):
        torch = _torch()
        if not (p.is_cuda and p.dtype == torch.float32 and p.is_contiguous() and p.numel() == self.param_count):
            raise ValueError(f"params must be a contiguous float32 CUDA vector of {self.param_count} entries")
        check(lib().t2s2_mlp_set_params(self._h, _ptr(p), _stream()))

    def forward(self, x):
        torch = _torch()
        _check(x, self.widths[0], "x")
        y = torch.empty(x.shape[0], self.widths[-1], dtype=torch.float32, device="cuda")
        check(lib().t2s2_mlp_forward(self._h, int(x.shape[0]), _ptr(x), _ptr(y), _stream()))
        return y

    def backward(self, x, dy):
        _check(x, self.widths[0], "x")
        _check(dy, self.widths[-1], "dy", x.shape[0])
        check(lib().t2s2_mlp_backward(self._h, int(x.shape[0]), _ptr(x), _ptr(dy), _stream()))

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        check(lib().t2s2_mlp_adam_step(self._h, float(lr), float(beta1), float(beta2), float(eps), _stream()))

    def infer_bf16(self, x):
        torch = _torch()
        _check(x, self.widths[0], "x")
        y = torch.empty(x.shape[0], self.widths[-1], dtype=torch.float32, device="cuda")
        check(lib().t2s2_mlp_infer_bf16(self._h, int(x.shape[0]), _ptr(x), _ptr(y), _stream()))
        return y

    def train(self, x, targets, n: Sequence[int], rank: int, epochs: int, batch: int, lr: float,
              seed: int = 0) -> List[float]:
        _check(x, self.widths[0], "x")
        _check(targets, self.widths[-1], "targets", x.shape[0])
        hist = (C.c_float * max(epochs, 1))()
        n_arr = (C.c_int * len(n))(*[int(v) for v in n])
        check(lib().t2s2_mlp_train(self._h, int(x.shape[0]), _ptr(x), _ptr(targets), len(n), n_arr, int(rank),
                                   int(epochs), int(batch), float(lr), C.c_ulonglong(seed), hist, _stream()))
        return [float(hist[i]) for i in range(epochs)]


def fit_loss(pred, target, n: Sequence[int], rank: int):
    """Per-sample gauge-invariant loss and its gradient (t2s2_tt_fit_loss)."""
    torch = _torch()
    size = flat_size(n, rank)
    _check(pred, size, "pred")
    _check(target, size, "target", pred.shape[0])
    B = int(pred.shape[0])
    loss = torch.empty(B, dtype=torch.float32, device="cuda")
    dpred = torch.empty_like(pred)
    n_arr = (C.c_int * len(n))(*[int(v) for v in n])
    check(lib().t2s2_tt_fit_loss(B, len(n), n_arr, int(rank), _ptr(pred), _ptr(target), _ptr(loss), _ptr(dpred),
                                 _stream()))
    return loss, dpred


def pack(x, rank: int, canonical: bool = True):
    """TT (FP64, ranks <= rank) -> flat FP32 vector (t2s2_tt_pack)."""
    torch = _torch()
    out = torch.empty(flat_size(x.n, rank), dtype=torch.float32, device="cuda")
    xs = x._struct()
    check(lib().t2s2_tt_pack(C.byref(xs), int(rank), int(bool(canonical)), _ptr(out), _stream()))
    return out


def unpack(y, n: Sequence[int], rank: int, cap: Optional[int] = None):
    """Flat FP32 vector -> TT with FP64 cores of rank `rank` (t2s2_tt_unpack);
    with cap, the core buffers are sized for a solve at that rank cap."""
    from . import TT
    if not (y.is_cuda and y.is_contiguous() and y.numel() == flat_size(n, rank)):
        raise ValueError("y must be a contiguous CUDA vector of the flat TT size")
    x = TT.empty(n, max(cap or rank, rank))
    xs = x._struct()
    n_arr = (C.c_int * len(n))(*[int(v) for v in n])
    check(lib().t2s2_tt_unpack(len(n), n_arr, int(rank), _ptr(y), C.byref(xs), _stream()))
    x._read_ranks()
    return x


def solution_target(problem, x, rank: int):
    """Training target of a solved instance: the solution rounded to rank
    `rank` (t2s2_tt_round, left-orthonormal cores) packed with canonical signs."""
    from . import TT
    y = TT.from_numpy(x.to_numpy())
    problem.tt_round(y, 1e-14, rank)
    return pack(y, rank, canonical=True)
