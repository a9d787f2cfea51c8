"""Seeded synthetic problem parameters shared by the oracle and the HIP path.

This module only draws and names numbers (advection fields, diffusion
coefficients, source parameters, grid sizes).  It holds none of the method's
arithmetic: no nodes, no operators, no source sampling.  Each side evaluates
the source on its own collocation grid.

Problem statement followed (Eq. advection-diffusion; Eq. pblm:time:A/B):
    -eps Lap u + beta . grad u = f  in [-1,1]^d,   u = g on the boundary,
with constant eps > 0 and constant beta.  The paper's experiments use
analytic or manufactured data only; these generators stand in for them:

* ``manufactured_sin_exp`` -- u = prod_i sin(pi x_i) exp(x_i) (vanishes on
  the boundary, so g = 0), used for the 2D N = 16 plain-method case.
* ``gaussian_mixture``     -- f = sum_m a_m prod_l exp(-(x_l - c_ml)^2 /
  (2 s_m^2)), a separable source of exact TT rank equal to the number of
  terms, a_m ~ U[0.5, 1.5], c_ml ~ U[-0.5, 0.5], s_m ~ U[0.2, 0.5];
  beta is drawn uniformly on the unit sphere (normalised Gaussian vector).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class GaussianMixture:
    """Parameters of f(x) = sum_m amp[m] * prod_l exp(-(x_l - centre[m,l])^2 / (2 width[m]^2))."""
    amp: np.ndarray      # (s,)
    centre: np.ndarray   # (s, d)
    width: np.ndarray    # (s,)

    @property
    def rank(self) -> int:
        return int(self.amp.size)


@dataclass
class Problem:
    """One steady advection-diffusion instance on [-1,1]^d with g = 0."""
    name: str
    d: int
    N: List[int]              # nodes per dimension (degree N-1)
    eps: float
    beta: np.ndarray          # (d,)
    scheme: int               # 1 = superconsistent, 0 = plain collocation
    tol: float                # TT truncation tolerance
    rank_cap: int
    source: str               # "sin_exp" or "gauss"
    gauss: Optional[GaussianMixture] = None
    target_residual: float = 1e-8
    seed: int = 0
    meta: dict = field(default_factory=dict)


def unit_vector(rng: np.random.Generator, d: int) -> np.ndarray:
    v = rng.standard_normal(d)
    return v / np.linalg.norm(v)


def gaussian_mixture(rng: np.random.Generator, d: int, s: int) -> GaussianMixture:
    amp = rng.uniform(0.5, 1.5, size=s)
    centre = rng.uniform(-0.5, 0.5, size=(s, d))
    width = rng.uniform(0.2, 0.5, size=s)
    return GaussianMixture(amp=amp, centre=centre, width=width)


def manufactured_2d(N: int = 16) -> Problem:
    """2D, beta = (1, 0.5), eps = 1e-2, u = prod sin(pi x) exp(x), TT tol 1e-12."""
    return Problem(name=f"2d_N{N}_manufactured", d=2, N=[N, N], eps=1e-2,
                   beta=np.array([1.0, 0.5]), scheme=1, tol=1e-12, rank_cap=N,
                   source="sin_exp", target_residual=1e-10)


def gauss_problem(d: int, N, eps: float, s: int, seed: int, tol: float,
                  rank_cap: int, scheme: int = 1, target_residual: float = 1e-8,
                  name: Optional[str] = None) -> Problem:
    rng = np.random.default_rng(seed)
    beta = unit_vector(rng, d)
    gm = gaussian_mixture(rng, d, s)
    Ns = [int(N)] * d if np.isscalar(N) else [int(v) for v in N]
    return Problem(name=name or f"{d}d_N{Ns[0]}_gauss{s}_seed{seed}", d=d, N=Ns,
                   eps=float(eps), beta=beta, scheme=scheme, tol=tol,
                   rank_cap=rank_cap, source="gauss", gauss=gm,
                   target_residual=target_residual, seed=seed)


def transport_3d(seed: int = 0) -> Problem:
    """3D, N = 32, eps/|beta L| = 1e-3 (L = 2, |beta| = 1 -> eps = 2e-3),
    4-Gaussian source, TT tol 1e-10, rank cap 32."""
    return gauss_problem(3, 32, 2e-3, 4, seed, tol=1e-10, rank_cap=32,
                         target_residual=1e-8, name=f"3d_N32_gauss4_seed{seed}")


def steady_6d(seed: int = 0, N: int = 32) -> Problem:
    """6D, N = 32 (32^6 grid, never formed), eps = 1e-3, rank-8 Gaussian source,
    target relative residual 1e-8."""
    return gauss_problem(6, N, 1e-3, 8, seed, tol=1e-9, rank_cap=160,
                         target_residual=1e-8, name=f"6d_N{N}_gauss8_seed{seed}")


def batched_instances(count: int = 256, base_seed: int = 0) -> List[Problem]:
    """Uneven instances: d ~ U{4,5,6}, N_l ~ U[16,48] per dimension,
    eps log-uniform in [1e-4, 1e-1], beta uniform on the sphere, rank-4
    Gaussian sources; solved to residual 1e-8 (TT tolerance 1e-10) under a
    rank cap of 128."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        d = int(rng.integers(4, 7))
        N = [int(v) for v in rng.integers(16, 49, size=d)]
        eps = float(10.0 ** rng.uniform(-4, -1))
        beta = unit_vector(rng, d)
        gm = gaussian_mixture(rng, d, 4)
        out.append(Problem(name=f"batch_{i}", d=d, N=N, eps=eps, beta=beta, scheme=1,
                           tol=1e-10, rank_cap=128, source="gauss", gauss=gm,
                           target_residual=1e-8, seed=base_seed + i))
    return out


# ---------------------------------------------------------------- learned warm start
WARM_D, WARM_N, WARM_SOURCES = 7, 24, 4
WARM_DIRECTION_SEED = 7_000_003


def warm_directions(d: int = WARM_D) -> np.ndarray:
    """The 4 fixed unit directions u_m in R^d along which the Gaussian centres move."""
    rng = np.random.default_rng(WARM_DIRECTION_SEED + d)
    return np.stack([unit_vector(rng, d) for _ in range(WARM_SOURCES)])


def warm_params(seed: int, d: int = WARM_D) -> dict:
    """Parameters of one learned-warm-start instance: beta on the unit sphere
    of R^d (d = 7), eps log-uniform in [1e-4, 1e-2], and 12 source
    parameters: per Gaussian m an amplitude a_m ~ U[0.5, 1.5], a width
    s_m ~ U[0.2, 0.5] and a signed offset t_m ~ U[-0.5, 0.5] of its centre
    t_m u_m along the fixed direction u_m."""
    rng = np.random.default_rng(seed)
    beta = unit_vector(rng, d)
    eps = float(10.0 ** rng.uniform(-4, -2))
    amp = rng.uniform(0.5, 1.5, size=WARM_SOURCES)
    width = rng.uniform(0.2, 0.5, size=WARM_SOURCES)
    offset = rng.uniform(-0.5, 0.5, size=WARM_SOURCES)
    return {"beta": beta, "eps": eps, "amp": amp, "width": width, "offset": offset}


def warm_instance(seed: int, d: int = WARM_D, N: int = WARM_N) -> Problem:
    """The instance of warm_params(seed, d) as a Problem on N nodes per
    dimension (7D, N = 24 for the learned warm start), solved to residual
    1e-8 with TT tolerance 1e-10 under rank cap 128."""
    q = warm_params(seed, d)
    centre = q["offset"][:, None] * warm_directions(d)
    gm = GaussianMixture(amp=q["amp"], centre=centre, width=q["width"])
    return Problem(name=f"warm{d}d_N{N}_{seed}", d=d, N=[N] * d, eps=q["eps"], beta=q["beta"], scheme=1,
                   tol=1e-10, rank_cap=128, source="gauss", gauss=gm, target_residual=1e-8, seed=seed,
                   meta={"params": q})


def dirichlet_problem(d: int, N, eps: float, seed: int, kind: str = "exp", rank_cap: int = 32) -> Problem:
    """Separable exact solution u = prod_l u_l(x_l) that does not vanish on the
    boundary (Dirichlet data g = u there), drawn from a seed.

    kind "poly": u_l a polynomial of degree N_l - 1 with Legendre coefficients
    ~ U[-1, 1] (the collocation solution then equals u at the GLL nodes);
    kind "exp":  u_l(x) = b_l exp(a_l x), a_l ~ U[-1.5, 1.5], b_l ~ U[0.5, 1.5].
    beta is uniform on the unit sphere.  Parameters only: the source and the
    boundary values are evaluated by each side on its own grids."""
    rng = np.random.default_rng(seed)
    Ns = [int(N)] * d if np.isscalar(N) else [int(v) for v in N]
    beta = unit_vector(rng, d)
    if kind == "poly":
        meta = {"kind": "poly", "coef": [rng.uniform(-1.0, 1.0, size=n) for n in Ns]}
    elif kind == "exp":
        meta = {"kind": "exp", "a": rng.uniform(-1.5, 1.5, size=d), "b": rng.uniform(0.5, 1.5, size=d)}
    else:
        raise ValueError(kind)
    return Problem(name=f"{d}d_N{Ns[0]}_dirichlet_{kind}_seed{seed}", d=d, N=Ns, eps=eps, beta=beta, scheme=1,
                   tol=1e-12, rank_cap=rank_cap, source="dirichlet", seed=seed, meta=meta)
