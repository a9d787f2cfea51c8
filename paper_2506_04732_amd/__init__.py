"""MI355X-native tensor-train solver for superconsistent spectral collocation (T^2S^2).

Thin Python binding of libt2s2 (C ABI in include/t2s2.h): argument
marshalling only.  Every step of the solve runs in the library's HIP kernels;
PyTorch provides device memory and the stream.  There is no CPU fallback:
without the built library every entry point raises ``LibraryMissing``.

Names follow the C ABI: ``nodes``, ``matrices_1d``, ``Problem`` (create /
operator / colloc / tt_matvec / tt_norm / tt_residual_norm / tt_round /
solve), ``solve_batched`` and ``local_solve``.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (PRECISION_FP64, PRECISION_MIXED, SCHEME_PLAIN, SCHEME_SC, T2S2_EFACTOR, T2S2_EINVAL,
                   T2S2_ENOTCONV, LibraryMissing,
                   T2S2Error, check, lib)

__all__ = ["nodes", "matrices_1d", "TT", "Problem", "MolProblem", "SpaceTimeProblem", "SolveResult", "solve_batched",
           "local_solve",
           "SCHEME_PLAIN",
           "SCHEME_SC",
           "PRECISION_FP64", "PRECISION_MIXED",
           "LibraryMissing", "T2S2Error", "lib"]


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def nodes(N: int, eps: float, beta: float, scheme: int = SCHEME_SC):
    """(GLL nodes (N,), collocation nodes (N-2,)) from the host builder."""
    x = np.empty(N)
    th = np.empty(N - 2)
    check(lib().t2s2_nodes(int(N), float(eps), float(beta), int(scheme), _dptr(x), _dptr(th)))
    return x, th


def matrices_1d(N: int, eps: float, beta: float, scheme: int = SCHEME_SC):
    """(E, D1, D2), each (N-2) x N: Lagrange basis of the GLL grid at the collocation nodes."""
    E = np.empty((N - 2, N))
    D1 = np.empty((N - 2, N))
    D2 = np.empty((N - 2, N))
    check(lib().t2s2_matrices_1d(int(N), float(eps), float(beta), int(scheme), _dptr(E), _dptr(D1), _dptr(D2)))
    return E, D1, D2


def timing_enable(on: bool = True) -> None:
    """Start (reset) or stop per-kernel-class event timing inside the library."""
    check(lib().t2s2_timing_enable(1 if on else 0))


def timing_classes(names=None) -> None:
    """Record only the named kernel classes while timing is on (None: all)."""
    if names is None:
        mask = 0xFFFFFFFF
    else:
        mask = 0
        for nm in names:
            mask |= 1 << _lib.TIMING_CLASSES.index(nm)
    check(lib().t2s2_timing_classes(mask))


def timing_read() -> dict:
    """{class name: {"ms", "launches", "bytes", "flops"}} accumulated since timing_enable(True)."""
    out = {}
    for cls, name in enumerate(_lib.TIMING_CLASSES):
        ms, n, b, f = C.c_double(), C.c_longlong(), C.c_double(), C.c_double()
        check(lib().t2s2_timing_read(cls, C.byref(ms), C.byref(n), C.byref(b), C.byref(f)))
        out[name] = {"ms": ms.value, "launches": int(n.value), "bytes": b.value, "flops": f.value}
    return out


def _torch():
    import torch
    return torch


class TT:
    """TT vector with device cores in caller-owned torch buffers.

    ``bufs[l]`` is a flat float64 CUDA tensor of at least ranks[l]*n[l]*ranks[l+1]
    elements (its capacity may be larger); ``core(l)`` views the live part.
    """

    def __init__(self, n: Sequence[int], ranks: Sequence[int], bufs):
        self.n = [int(v) for v in n]
        self.ranks = [int(v) for v in ranks]
        self.bufs = list(bufs)
        self.d = len(self.n)

    @staticmethod
    def empty(n: Sequence[int], cap: int, device="cuda"):
        torch = _torch()
        d = len(n)
        caps = [1] + [cap] * (d - 1) + [1]
        bufs = [torch.zeros(caps[l] * n[l] * caps[l + 1], dtype=torch.float64, device=device) for l in range(d)]
        return TT(n, [1] * (d + 1), bufs)

    @staticmethod
    def empty_like_ranks(n: Sequence[int], ranks: Sequence[int], device="cuda"):
        torch = _torch()
        bufs = [torch.zeros(ranks[l] * n[l] * ranks[l + 1], dtype=torch.float64, device=device)
                for l in range(len(n))]
        return TT(n, ranks, bufs)

    @staticmethod
    def from_numpy(cores: Sequence[np.ndarray], device="cuda", cap: Optional[int] = None):
        torch = _torch()
        n = [c.shape[1] for c in cores]
        ranks = [cores[0].shape[0]] + [c.shape[2] for c in cores]
        bufs = []
        for l, c in enumerate(cores):
            size = c.size
            if cap is not None:
                r0 = 1 if l == 0 else cap
                r1 = 1 if l == len(cores) - 1 else cap
                size = max(size, r0 * c.shape[1] * r1)
            b = torch.zeros(size, dtype=torch.float64, device=device)
            b[:c.size] = torch.from_numpy(np.ascontiguousarray(c, dtype=np.float64).ravel()).to(device)
            bufs.append(b)
        return TT(n, ranks, bufs)

    def core(self, l: int):
        r0, n, r1 = self.ranks[l], self.n[l], self.ranks[l + 1]
        return self.bufs[l][: r0 * n * r1].view(r0, n, r1)

    def to_numpy(self) -> List[np.ndarray]:
        return [self.core(l).detach().cpu().numpy().copy() for l in range(self.d)]

    def _struct(self):
        self._n_arr = (C.c_int * self.d)(*self.n)
        self._r_arr = (C.c_int * (self.d + 1))(*self.ranks)
        self._c_arr = (C.c_void_p * self.d)(*[b.data_ptr() for b in self.bufs])
        return _lib.TTStruct(self.d, self._n_arr, self._r_arr, self._c_arr)

    def _read_ranks(self):
        self.ranks = [int(self._r_arr[i]) for i in range(self.d + 1)]


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class SolveResult:
    x: TT
    status: int
    sweeps: int
    residual: float
    ranks: List[int]
    time_ms: float
    history_residual: List[float] = field(default_factory=list)
    history_local: List[float] = field(default_factory=list)
    history_max_rank: List[int] = field(default_factory=list)
    history_time_ms: List[float] = field(default_factory=list)
    precision: int = PRECISION_FP64
    local_systems: int = 0
    refinement_steps: int = 0
    fp64_fallbacks: int = 0
    warm_start_used: int = 0
    warm_residual: float = -1.0
    cold_residual: float = -1.0
    refinement_capped: int = 0
    max_eig_cond: float = 0.0
    phase_ms: dict = field(default_factory=dict)

    @property
    def converged(self) -> bool:
        return self.status == 0


class Problem:
    """-eps Lap u + beta . grad u + rho u = f on [-1,1]^d, u = g on the boundary
    (t2s2_problem_create, or t2s2_problem_create_reaction for rho != 0)."""

    def __init__(self, d: int, N, eps: float, beta, scheme: int = SCHEME_SC, rank_cap: int = 64,
                 rho: float = 0.0, _mol=None):
        Ns = [int(N)] * d if np.isscalar(N) else [int(v) for v in N]
        self.d, self.N, self.eps, self.scheme, self.rank_cap = d, Ns, float(eps), int(scheme), int(rank_cap)
        self.beta = np.asarray(beta, dtype=np.float64).copy()
        self.rho = float(rho)
        self.m = [v - 2 for v in Ns]
        h = C.c_void_p()
        n_arr = (C.c_int * d)(*Ns)
        b_arr = self.beta.ctypes.data_as(C.POINTER(C.c_double))
        if _mol is not None:
            dt, theta = _mol
            check(lib().t2s2_mol_create(d, n_arr, self.eps, b_arr, self.rho, float(dt), float(theta), self.scheme,
                                        self.rank_cap, C.byref(h)))
        elif self.rho != 0.0:
            check(lib().t2s2_problem_create_reaction(d, n_arr, self.eps, b_arr, self.rho, self.scheme,
                                                     self.rank_cap, C.byref(h)))
        else:
            check(lib().t2s2_problem_create(d, n_arr, self.eps, b_arr, self.scheme, self.rank_cap, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().t2s2_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- queries
    def colloc(self, l: int) -> np.ndarray:
        th = np.empty(self.m[l])
        check(lib().t2s2_problem_colloc(self._h, int(l), _dptr(th)))
        return th

    def operator(self) -> _lib.TTMStruct:
        s = _lib.TTMStruct()
        check(lib().t2s2_problem_operator(self._h, C.byref(s)))
        return s

    def operator_ranks(self) -> List[int]:
        s = self.operator()
        return [int(s.ranks[i]) for i in range(self.d + 1)]

    # ---------------------------------------------------------- building blocks
    def tt_matvec(self, x: TT) -> TT:
        op = self.operator()
        R = [int(op.ranks[i]) for i in range(self.d + 1)]
        y = TT.empty_like_ranks(x.n, [R[i] * x.ranks[i] for i in range(self.d + 1)])
        xs, ys = x._struct(), y._struct()
        check(lib().t2s2_tt_matvec(C.byref(op), C.byref(xs), C.byref(ys), _stream()))
        y._read_ranks()
        return y

    def tt_matvec_noalloc(self, x: TT, out: Optional[TT] = None) -> TT:
        """t2s2_tt_matvec_noalloc with this problem's operator (out: caller's
        buffers, e.g. preallocated for graph capture)."""
        op = self.operator()
        return ttm_matvec(op, x, out=out, noalloc=True)

    def tt_fiber(self, x: TT, l: int, idx) -> np.ndarray:
        """t2s2_tt_fiber: x along mode l through the indices idx (idx[l] ignored)."""
        torch = _torch()
        out = torch.empty(x.n[l], dtype=torch.float64, device="cuda")
        arr = (C.c_int * x.d)(*[int(v) for v in idx])
        xs = x._struct()
        check(lib().t2s2_tt_fiber(self._h, C.byref(xs), int(l), arr, C.c_void_p(out.data_ptr()), _stream()))
        return out.cpu().numpy()

    def tt_norm(self, x: TT) -> float:
        out = C.c_double()
        xs = x._struct()
        check(lib().t2s2_tt_norm(self._h, C.byref(xs), C.byref(out), _stream()))
        return out.value

    def tt_residual_norm(self, x: TT, f: TT) -> float:
        out = C.c_double()
        xs, fs = x._struct(), f._struct()
        check(lib().t2s2_tt_residual_norm(self._h, C.byref(xs), C.byref(fs), C.byref(out), _stream()))
        return out.value

    def tt_round(self, x: TT, tol: float, rmax: int = 10 ** 6) -> TT:
        xs = x._struct()
        check(lib().t2s2_tt_round(self._h, C.byref(xs), float(tol), int(rmax), _stream()))
        x._read_ranks()
        return x

    # ------------------------------------------------------------------ solve
    def solve(self, f: TT, x0: Optional[TT] = None, *, g: Optional[TT] = None, tol: float = 1e-10,
              target: float = 1e-8, max_sweeps: int = 40, kick: int = 8, rank_cap: Optional[int] = None,
              init_rank: int = 2, seed: int = 0, check_every: int = 1, verbose: bool = False,
              out: Optional[TT] = None, precision: int = PRECISION_FP64,
              warm_judge: bool = False, overlap: bool = True) -> SolveResult:
        """t2s2_solve.  f on the collocation grid (modes N_l - 2); g optional
        Dirichlet data on the GLL grid (modes N_l); the result holds the
        interior values."""
        cap = int(rank_cap or self.rank_cap)
        x = out if out is not None else TT.empty(self.m, cap)
        o = _options(tol, target, max_sweeps, kick, cap, init_rank, seed, check_every, verbose, precision)
        o.warm_judge = int(bool(warm_judge))
        o.overlap = int(bool(overlap))
        rep = _lib.Report()
        fs, xs = f._struct(), x._struct()
        x0s = x0._struct() if x0 is not None else None
        gs = g._struct() if g is not None else None
        code = lib().t2s2_solve(self._h, C.byref(fs), C.byref(gs) if gs is not None else None,
                                C.byref(x0s) if x0s is not None else None, C.byref(o),
                                C.byref(xs), C.byref(rep), _stream())
        check(code, allow=(T2S2_ENOTCONV,))
        x._read_ranks()
        return _result(x, code, rep, self.d)


class SpaceTimeProblem(Problem):
    """t2s2_problem_create_general: space dimensions x_l in [-1, 1] with variable
    separable advection beta_l(x_l) = sum_k coef[l][k] P_k(x_l) (Legendre
    series) and optionally the time dimension t in [0, T] (kind 1, the value
    at t = 0 given).  N, kinds: per dimension; beta_coefs: one coefficient
    list per space dimension, in order."""

    def __init__(self, N: Sequence[int], kinds: Sequence[int], eps: float, beta_coefs, T: float = 0.0,
                 rho: float = 0.0, scheme: int = SCHEME_SC, rank_cap: int = 64):
        d = len(N)
        self.d, self.N, self.eps, self.scheme, self.rank_cap = d, [int(v) for v in N], float(eps), int(scheme), \
            int(rank_cap)
        self.kinds, self.T, self.rho = [int(k) for k in kinds], float(T), float(rho)
        self.m = [n - 1 if k == 1 else n - 2 for n, k in zip(self.N, self.kinds)]
        coefs = [np.asarray(c, dtype=np.float64).ravel() for c in beta_coefs]
        nb = []
        it = iter(coefs)
        for k in self.kinds:
            nb.append(len(next(it)) if k == 0 else 0)
        flat = np.concatenate(coefs) if coefs else np.zeros(1)
        self.beta = None
        h = C.c_void_p()
        n_arr = (C.c_int * d)(*self.N)
        k_arr = (C.c_int * d)(*self.kinds)
        nb_arr = (C.c_int * d)(*nb)
        check(lib().t2s2_problem_create_general(d, n_arr, k_arr, self.eps, flat.ctypes.data_as(C.POINTER(C.c_double)),
                                                nb_arr, self.rho, self.T, self.scheme, self.rank_cap, C.byref(h)))
        self._h = h


class MolProblem(Problem):
    """Method of lines (t2s2_mol_create / t2s2_mol_step): theta-scheme steps of
    du/dt - eps Lap u + beta . grad u + rho u = b, u = 0 on the boundary;
    theta = 1 backward Euler, 1/2 Crank-Nicolson."""

    def __init__(self, d: int, N, eps: float, beta, dt: float, theta: float = 0.5, rho: float = 0.0,
                 scheme: int = SCHEME_SC, rank_cap: int = 64):
        self.dt, self.theta = float(dt), float(theta)
        super().__init__(d, N, eps, beta, scheme, rank_cap, rho=rho, _mol=(dt, theta))

    def step(self, u: TT, b: Optional[TT] = None, *, tol: float = 1e-10, target: float = 1e-8,
             max_sweeps: int = 40, kick: int = 8, rank_cap: Optional[int] = None, check_every: int = 1,
             out: Optional[TT] = None, precision: int = PRECISION_FP64, overlap: bool = True) -> SolveResult:
        """One step from u (interior values); b: the step's source at the collocation nodes."""
        cap = int(rank_cap or self.rank_cap)
        x = out if out is not None else TT.empty(self.m, cap)
        o = _options(tol, target, max_sweeps, kick, cap, 1, 0, check_every, False, precision)
        o.overlap = int(bool(overlap))
        rep = _lib.Report()
        us, xs = u._struct(), x._struct()
        bs = b._struct() if b is not None else None
        code = lib().t2s2_mol_step(self._h, C.byref(us), C.byref(bs) if bs is not None else None, C.byref(o),
                                   C.byref(xs), C.byref(rep), _stream())
        check(code, allow=(T2S2_ENOTCONV,))
        x._read_ranks()
        return _result(x, code, rep, self.d)


def _options(tol, target, max_sweeps, kick, cap, init_rank, seed, check_every, verbose, precision):
    o = _lib.Options()
    lib().t2s2_default_options(C.byref(o))
    o.tol, o.target, o.max_sweeps, o.kick = float(tol), float(target), int(max_sweeps), int(kick)
    o.rank_cap, o.init_rank, o.seed = int(cap), int(init_rank), int(seed)
    o.check_every, o.verbose = int(check_every), int(bool(verbose))
    o.precision = int(precision)
    return o


def _result(x: TT, code: int, rep, d: int) -> SolveResult:
    h = rep.history_len
    return SolveResult(x=x, status=rep.status if code in (0, T2S2_ENOTCONV) else code, sweeps=rep.sweeps,
                       residual=rep.residual, ranks=list(rep.ranks[: d + 1]), time_ms=rep.time_ms,
                       history_residual=list(rep.history_residual[:h]),
                       history_local=list(rep.history_local[:h]),
                       history_max_rank=list(rep.history_max_rank[:h]),
                       history_time_ms=list(rep.history_time_ms[:h]), precision=rep.precision,
                       local_systems=rep.local_systems, refinement_steps=rep.refinement_steps,
                       fp64_fallbacks=rep.fp64_fallbacks, warm_start_used=rep.warm_start_used,
                       warm_residual=rep.warm_residual, cold_residual=rep.cold_residual,
                       refinement_capped=rep.refinement_capped, max_eig_cond=rep.max_eig_cond,
                       phase_ms={n: rep.phase_ms[i] for i, n in enumerate(_lib.PHASE_NAMES)})


def solve_batched(problems: Sequence["Problem"], fs: Sequence[TT], *, x0s: Optional[Sequence[Optional[TT]]] = None,
                  gs: Optional[Sequence[Optional[TT]]] = None,
                  outs: Optional[Sequence[TT]] = None, workers: int = 16, tol: float = 1e-10,
                  target: float = 1e-8, max_sweeps: int = 40, kick: int = 8, rank_cap: Optional[int] = None,
                  init_rank: int = 2, seed: int = 0, check_every: int = 1,
                  precision: int = PRECISION_FP64, overlap: bool = False) -> List[SolveResult]:
    """t2s2_solve_batched: every instance solved as Problem.solve would, up to
    `workers` at a time on their own streams.  rank_cap None: each problem's own."""
    count = len(problems)
    if len(fs) != count or any(v is not None and len(v) != count for v in (x0s, gs, outs)):
        raise ValueError("problems, fs, gs, x0s and outs must have the same length")
    if count == 0:
        return []
    caps = [int(rank_cap or p.rank_cap) for p in problems]
    if len(set(caps)) != 1:
        raise ValueError("one rank_cap applies to every instance: pass rank_cap or use equal problem caps")
    xs = list(outs) if outs is not None else [TT.empty(p.m, caps[0]) for p in problems]
    o = _options(tol, target, max_sweeps, kick, caps[0], init_rank, seed, check_every, False, precision)
    o.overlap = int(bool(overlap))
    reps = (_lib.Report * count)()
    fst = [f._struct() for f in fs]
    xst = [x._struct() for x in xs]
    ttp = C.POINTER(_lib.TTStruct)
    f_arr = (ttp * count)(*[C.pointer(v) for v in fst])
    x_arr = (ttp * count)(*[C.pointer(v) for v in xst])
    x0_arr = None
    if x0s is not None:
        x0st = [x0._struct() if x0 is not None else None for x0 in x0s]
        x0_arr = (ttp * count)(*[C.pointer(v) if v is not None else ttp() for v in x0st])
    g_arr = None
    if gs is not None:
        gst = [g._struct() if g is not None else None for g in gs]
        g_arr = (ttp * count)(*[C.pointer(v) if v is not None else ttp() for v in gst])
    h_arr = (C.c_void_p * count)(*[p._h.value for p in problems])
    code = lib().t2s2_solve_batched(count, h_arr, f_arr, g_arr, x0_arr, C.byref(o), x_arr, reps, int(workers),
                                    _stream())
    check(code, allow=(T2S2_ENOTCONV,))
    out = []
    for i, x in enumerate(xs):
        x._read_ranks()
        out.append(_result(x, code, reps[i], problems[i].d))
    return out


def ttm_matvec(op: "_lib.TTMStruct", x: TT, out: Optional[TT] = None, noalloc: bool = False) -> TT:
    """y = A x for a TT-matrix descriptor (t2s2_tt_matvec / _noalloc)."""
    d = x.d
    R = [int(op.ranks[i]) for i in range(d + 1)]
    y = out if out is not None else TT.empty_like_ranks(x.n, [R[i] * x.ranks[i] for i in range(d + 1)])
    xs, ys = x._struct(), y._struct()
    fn = lib().t2s2_tt_matvec_noalloc if noalloc else lib().t2s2_tt_matvec
    check(fn(C.byref(op), C.byref(xs), C.byref(ys), _stream()))
    y._read_ranks()
    return y


def debug_iteration_limits(francis_steps: int = 0, jacobi_sweeps: int = 0) -> None:
    """t2s2_debug_iteration_limits (0 restores the defaults)."""
    check(lib().t2s2_debug_iteration_limits(int(francis_steps), int(jacobi_sweeps)))


LOCAL_EIG, LOCAL_HESS, LOCAL_HESS_RIGHT = 0, 1, 2


def local_solve(Lint, K, Rint, g, method: int = LOCAL_HESS):
    """t2s2_local_solve: u = (Lint (+) K (+) Rint)^{-1} g for g of shape
    (r1, m, r2); all arguments float64 CUDA tensors.  Returns u (new tensor)."""
    torch = _torch()
    mats = [Lint, K, Rint, g]
    for a in mats:
        if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float64 and a.is_contiguous()):
            raise TypeError("local_solve: arguments must be contiguous float64 CUDA tensors")
    r1, m, r2 = g.shape
    if Lint.shape != (r1, r1) or K.shape != (m, m) or Rint.shape != (r2, r2):
        raise ValueError("local_solve: Lint (r1 x r1), K (m x m), Rint (r2 x r2) must match g (r1, m, r2)")
    u = torch.empty_like(g)
    check(lib().t2s2_local_solve(r1, m, r2, C.c_void_p(Lint.data_ptr()), C.c_void_p(K.data_ptr()),
                                 C.c_void_p(Rint.data_ptr()), C.c_void_p(g.data_ptr()), C.c_void_p(u.data_ptr()),
                                 int(method), _stream()))
    return u
