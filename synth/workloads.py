"""Seeded workload generators (numpy PCG64 only; no solver arithmetic).

Conventions shared by every consumer of these arrays
----------------------------------------------------
* Space: the unit interval/square/cube with ``n`` interior nodes per axis,
  spacing ``h = 1/(n+1)``; node ``i`` (0..n+1) sits at ``x = i*h``.  Nodes 0 and
  n+1 are on the Dirichlet boundary.  Array axes are ordered (z, y, x): the
  last axis is x and is the fastest-varying one in memory.
* Time: ``N`` steps; uniform (length ``tau = T/N``, step ``n`` (1..N) ends at
  ``t_n = n*tau``) unless ``steps`` holds the lengths tau_n (summing to T), when
  ``t_n = tau_1 + ... + tau_n``.  Index ``n-1`` of every time axis below refers
  to ``t_n``.  ``tau`` is always T/N (the mean step).
* Coefficient: ``kappa(t_n, x) = sum_r tcoef[r, n-1] * kfields[r](x)``, the
  fields sampled on all ``(n+2)^d`` nodes including the boundary.
* Source ``F[n-1]`` is the source at ``t_n`` on the interior nodes; ``u0`` is
  the initial datum on the interior nodes.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Problem:
    dim: int
    n: int
    N: int
    T: float
    kfields: np.ndarray  # (R,) + (n+2,)*dim
    tcoef: np.ndarray    # (R, N)
    F: np.ndarray        # (N,) + (n,)*dim
    u0: np.ndarray       # (n,)*dim
    name: str = ""
    seed: int = 0
    steps: np.ndarray | None = None   # (N,) step lengths; None: uniform

    @property
    def tau(self) -> float:
        return self.T / self.N

    @property
    def taus(self) -> np.ndarray:
        return np.full(self.N, self.T / self.N) if self.steps is None else self.steps

    @property
    def h(self) -> float:
        return 1.0 / (self.n + 1)

    @property
    def R(self) -> int:
        return self.kfields.shape[0]

    @property
    def npts(self) -> int:
        return self.n ** self.dim

    @property
    def dofs(self) -> int:
        return self.N * self.npts


def _nodes(n: int) -> np.ndarray:
    return np.arange(n + 2, dtype=np.float64) / (n + 1)


def _interior(n: int) -> np.ndarray:
    return np.arange(1, n + 1, dtype=np.float64) / (n + 1)


def _times(N: int, T: float, steps=None) -> np.ndarray:
    if steps is not None:
        return np.cumsum(steps)
    return T * np.arange(1, N + 1, dtype=np.float64) / N


def graded_steps(N: int, T: float = 1.0, ratio: float = 8.0, jitter: float = 0.0, seed: int = 0) -> np.ndarray:
    """N step lengths growing geometrically from the first to the last by
    ``ratio`` (small steps first, as for rough initial data), each optionally
    scaled by a factor uniform in [1 - jitter, 1 + jitter], normalised to sum T."""
    q = ratio ** (np.arange(N, dtype=np.float64) / max(N - 1, 1))
    if jitter > 0:
        q = q * np.random.default_rng(seed).uniform(1 - jitter, 1 + jitter, N)
    return T * q / q.sum()


def _outer(vecs):
    """Tensor product of 1-D arrays; vecs ordered (x, y, z) -> array (z, y, x)."""
    out = vecs[0]
    for v in vecs[1:]:
        out = np.multiply.outer(v, out)
    return out


def sine_modes(n: int, dim: int, kmax: int, rng: np.random.Generator) -> np.ndarray:
    """sum over k_1..k_d <= kmax of c_k prod_a sin(k_a pi x_a), c_k ~ N(0,1)."""
    x = _interior(n)
    kk = np.arange(1, kmax + 1)
    S = np.sin(np.pi * np.multiply.outer(kk, x))  # (kmax, n)
    c = rng.standard_normal((kmax,) * dim)        # axes (k_z, k_y, k_x)
    if dim == 1:
        return c @ S
    if dim == 2:
        return S.T @ c @ S                         # (y, x)
    return np.einsum("abc,ai,bj,ck->ijk", c, S, S, S, optimize=True)


def gaussian_factors(n: int, dim: int, N: int, T: float, rng: np.random.Generator,
                     count: int = 8):
    """Separable factors of ``count`` space-time Gaussians
    a_i exp(-|x-x_i|^2/2s_i^2 - (t-t_i)^2/2sig_i^2): a list of (g_t, [g_x, g_y, ...])
    with g_t of length N (amplitude included) and each g of length n.

    Draw order per Gaussian block: centres (dim space coords then t) ~ U[0,1]
    (t scaled by T), widths s ~ U[0.05,0.15], sig ~ U[0.1,0.3], amplitudes a ~ N(0,1).
    """
    centres = rng.uniform(0.0, 1.0, size=(count, dim + 1))
    s = rng.uniform(0.05, 0.15, size=count)
    sig = rng.uniform(0.1, 0.3, size=count)
    a = rng.standard_normal(count)
    x = _interior(n)
    t = _times(N, T)
    out = []
    for i in range(count):
        gx = [np.exp(-((x - centres[i, ax]) ** 2) / (2 * s[i] ** 2)) for ax in range(dim)]
        gt = a[i] * np.exp(-((t - T * centres[i, dim]) ** 2) / (2 * sig[i] ** 2))
        out.append((gt, gx))
    return out


def source_from_factors(factors, n: int, dim: int, N: int) -> np.ndarray:
    """F = sum_i g_t,i (x) (... (x) g_y,i (x) g_x,i), accumulated in factor order."""
    F = np.zeros((N,) + (n,) * dim)
    for gt, gx in factors:
        F += np.multiply.outer(gt, _outer(gx))
    return F


def gaussian_source(n: int, dim: int, N: int, T: float, rng: np.random.Generator,
                    count: int = 8) -> np.ndarray:
    """Sum of ``count`` space-time Gaussians (see ``gaussian_factors``)."""
    return source_from_factors(gaussian_factors(n, dim, N, T, rng, count), n, dim, N)


def lognormal_field(n: int, dim: int, ell: float, contrast: float,
                    rng: np.random.Generator) -> np.ndarray:
    """Lognormal field on the (n+2)^d nodes (boundary included).

    Gaussian field with squared-exponential covariance of length ``ell`` by
    spectral synthesis on a periodic grid twice as long per axis (to suppress
    wrap-around correlation), cropped, then affinely rescaled so that
    ``log kappa`` spans exactly ``[-ln(c)/2, ln(c)/2]``: max/min = contrast and
    geometric mid-range 1.
    """
    import scipy.fft as sfft

    m = n + 2
    M = 2 * m
    h = 1.0 / (n + 1)
    xi = rng.standard_normal((M,) * dim)
    Xf = sfft.rfftn(xi, workers=-1)
    del xi
    k_full = 2 * np.pi * np.fft.fftfreq(M, d=h)
    k_half = 2 * np.pi * np.fft.rfftfreq(M, d=h)
    k2 = k_half ** 2
    for ax in range(dim - 1):
        shape = [1] * dim
        shape[ax] = M
        k2 = k2 + (k_full ** 2).reshape(shape)
    Xf *= np.sqrt(np.exp(-0.5 * ell ** 2 * k2))
    g = sfft.irfftn(Xf, s=(M,) * dim, workers=-1)
    del Xf
    g = np.ascontiguousarray(g[(slice(0, m),) * dim])
    gmin, gmax = g.min(), g.max()
    g = (g - gmin) / (gmax - gmin) - 0.5
    return np.exp(g * math.log(contrast))


def manufactured_u(n: int, dim: int, N: int, T: float) -> np.ndarray:
    """u*(t,x) = exp(-d pi^2 t) prod sin(pi x_a) at t_0..t_N -> shape (N+1,)+(n,)*dim."""
    x = _interior(n)
    s = _outer([np.sin(np.pi * x)] * dim)
    t = T * np.arange(0, N + 1) / N
    return np.multiply.outer(np.exp(-dim * np.pi ** 2 * t), s)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def heat1d_random(n: int = 63, N: int = 64, T: float = 1.0, seed: int = 1001, steps=None) -> Problem:
    """1-D heat: kappa = 1 + 0.5 sin(2 pi t); F ~ N(0,1) per node and step;
    u0 = sin(pi x) + 0.1 N(0,1).  ``steps``: optional step lengths (sum T)."""
    rng = np.random.default_rng(seed)
    t = _times(N, T, steps)
    kf = np.ones((1, n + 2))
    tc = (1.0 + 0.5 * np.sin(2 * np.pi * t))[None, :]
    F = rng.standard_normal((N, n))
    u0 = np.sin(np.pi * _interior(n)) + 0.1 * rng.standard_normal(n)
    return Problem(1, n, N, T, kf, tc, F, u0, name="heat1d_random", seed=seed,
                   steps=None if steps is None else np.asarray(steps, dtype=np.float64))


def heat2d_parts(n: int = 255, N: int = 256, T: float = 1.0, seed: int = 1002,
                 phase: float | None = None, kmax: int = 16):
    """Everything of ``heat2d_gaussians`` except the assembled source: returns
    (kfields, tcoef, source factors, u0); ``source_from_factors`` gives F."""
    rng = np.random.default_rng(seed)
    t = _times(N, T)
    if phase is None:
        x = _nodes(n)
        kf = np.stack([np.ones((n + 2, n + 2)), np.broadcast_to(np.cos(np.pi * x), (n + 2, n + 2))])
        tc = np.stack([np.ones(N), 0.5 * np.sin(2 * np.pi * t)])
    else:
        kf = np.ones((1, n + 2, n + 2))
        tc = (1.0 + 0.5 * np.sin(2 * np.pi * t + phase))[None, :]
    factors = gaussian_factors(n, 2, N, T, rng)
    u0 = sine_modes(n, 2, min(kmax, n), rng)
    return np.ascontiguousarray(kf), tc, factors, u0


def heat2d_gaussians(n: int = 255, N: int = 256, T: float = 1.0, seed: int = 1002,
                     phase: float | None = None, kmax: int = 16) -> Problem:
    """2-D heat.  Default coefficient kappa = 1 + 0.5 sin(2 pi t) cos(pi x)
    (two separable terms); with ``phase`` given, kappa = 1 + 0.5 sin(2 pi t + phase)
    (one term).  F = 8 space-time Gaussians; u0 = random sine modes k <= kmax."""
    kf, tc, factors, u0 = heat2d_parts(n, N, T, seed, phase, kmax)
    F = source_from_factors(factors, n, 2, N)
    return Problem(2, n, N, T, kf, tc, F, u0, name="heat2d_gaussians", seed=seed)


def heat3d_lognormal(n: int = 127, N: int = 128, T: float = 1.0, seed: int = 1003,
                     contrast: float = 1e2, ell: float = 0.1, source: str = "gaussians") -> Problem:
    """3-D heat, kappa = kappa_s(x) (1 + 0.3 t) with kappa_s lognormal.

    ``source="gaussians"``: F = 8 space-time Gaussians, u0 = sin(pi x)sin(pi y)sin(pi z).
    ``source="none"``: F is None; callers build the manufactured source for
    u*(t,x) = exp(-3 pi^2 t) sin(pi x) sin(pi y) sin(pi z) (whose u0 this is),
    F_n = (u*_n - u*_{n-1}) / tau + A_n u*_n, which needs the spatial operator
    and so is not built here.
    """
    rng = np.random.default_rng(seed)
    t = _times(N, T)
    ks = lognormal_field(n, 3, ell, contrast, rng)[None]
    tc = (1.0 + 0.3 * t)[None, :]
    u0 = manufactured_u(n, 3, 1, T)[0]
    if source == "gaussians":
        F = gaussian_source(n, 3, N, T, rng)
    else:
        F = None
    return Problem(3, n, N, T, ks, tc, F, u0, name="heat3d_lognormal", seed=seed)


def batch2d(count: int = 64, seed: int = 1004, sides=(63, 127, 255, 511), nt_range=(32, 1024),
            side_cap: int | None = None, nt_cap: int | None = None):
    """Specs of a batch of independent 2-D problems (side, N, phase, seed).

    Returns a list of dicts; build each problem lazily with ``batch2d_problem``.
    ``side_cap``/``nt_cap`` clamp the draws (for small test batches) without
    changing the random stream.
    """
    rng = np.random.default_rng(seed)
    side = rng.choice(np.asarray(sides), size=count)
    nt = rng.integers(nt_range[0], nt_range[1] + 1, size=count)
    phase = rng.uniform(0.0, 2 * np.pi, size=count)
    specs = []
    for i in range(count):
        s = int(side[i]) if side_cap is None else min(int(side[i]), side_cap)
        N = int(nt[i]) if nt_cap is None else min(int(nt[i]), nt_cap)
        specs.append(dict(side=s, N=N, phase=float(phase[i]), seed=4000 + i))
    return specs


def batch2d_problem(spec) -> Problem:
    return heat2d_gaussians(n=spec["side"], N=spec["N"], seed=spec["seed"], phase=spec["phase"])


def batch2d_parts(spec):
    """``heat2d_parts`` of one batch problem (source left as factors)."""
    return heat2d_parts(n=spec["side"], N=spec["N"], seed=spec["seed"], phase=spec["phase"])


def small_problem(dim: int, n: int, N: int, seed: int = 7, T: float = 1.0, R: int = 2,
                  amp: float = 0.5, steps=None) -> Problem:
    """Small generic problem for unit and parity tests.

    kappa(t,x) = 1 + amp * sin(2 pi t + phi) * g(x) with g a rough random nodal
    field in [-1, 1] (R = 2 separable terms; R = 1 drops the second term and
    uses kappa = 1 + amp sin(2 pi t + phi); R = 3, 4 add R - 1 rough fields of
    weight 1/(R-1) with time frequencies 1 .. R-1).  kappa stays in [1-amp, 1+amp],
    as in the paper-style workloads.  F and u0 are standard normal.  ``steps``:
    optional step lengths (sum T).
    """
    rng = np.random.default_rng(seed)
    t = _times(N, T, steps)
    shape = (n + 2,) * dim
    phi = rng.uniform(0, 2 * np.pi)
    if R == 1:
        kf = np.ones((1,) + shape)
        tc = (1.0 + amp * np.sin(2 * np.pi * t + phi))[None, :]
    elif R == 2:
        g = rng.uniform(-1.0, 1.0, size=shape)
        kf = np.stack([np.ones(shape), g])
        tc = np.stack([np.ones(N), amp * np.sin(2 * np.pi * t + phi)])
    else:
        # R - 1 rough fields with time frequencies 1 .. R-1, each scaled by 1/(R-1)
        gs = [rng.uniform(-1.0, 1.0, size=shape) / (R - 1) for _ in range(R - 1)]
        phis = [phi] + list(rng.uniform(0, 2 * np.pi, size=R - 2))
        kf = np.stack([np.ones(shape)] + gs)
        tc = np.stack([np.ones(N)] + [amp * np.sin(2 * np.pi * (r + 1) * t + phis[r]) for r in range(R - 1)])
    F = rng.standard_normal((N,) + (n,) * dim)
    u0 = rng.standard_normal((n,) * dim)
    return Problem(dim, n, N, T, kf, tc, F, u0, name=f"small{dim}d", seed=seed,
                   steps=None if steps is None else np.asarray(steps, dtype=np.float64))


def heat2d_sine(n: int = 63, N: int = 512, T: float = 1.0) -> Problem:
    """The 2-D problem of the paper's robustness study (Section 8.2) in
    finite-difference form: kappa = 1, T = 1, F = 0, u0 = sin(pi x) sin(pi y);
    n = 2^k - 1 interior nodes per axis is the mesh h = 2^-k."""
    s = np.sin(np.pi * _interior(n))
    u0 = _outer([s, s])
    return Problem(2, n, N, T, np.ones((1, n + 2, n + 2)), np.ones((1, N)), np.zeros((N, n, n)), u0,
                   name="heat2d_sine", seed=0)


def heat3d_sine(n: int = 15, N: int = 16, T: float = 0.1) -> Problem:
    """The 3-D test problem of the paper's time-parallel experiments (Section
    8.3) in finite-difference form: kappa = 1, T = 0.1, exact solution
    exp(-3 pi^2 t) sin(pi x) sin(pi y) sin(pi z), which solves the heat equation
    with F = 0 and u0 = sin(pi x) sin(pi y) sin(pi z).  n = 15 interior nodes
    per axis is the paper's mesh of 16^3 cells (h = 1/16)."""
    x = _interior(n)
    s = np.sin(np.pi * x)
    u0 = _outer([s, s, s])
    kf = np.ones((1, n + 2, n + 2, n + 2))
    tc = np.ones((1, N))
    F = np.zeros((N, n, n, n))
    return Problem(3, n, N, T, kf, tc, F, u0, name="heat3d_sine", seed=0)


CONFIG_BUILDERS = {
    "heat1d_63_N64": lambda: heat1d_random(),
    "heat2d_255_N256": lambda: heat2d_gaussians(),
    "heat3d_127_N128_lognormal": lambda: heat3d_lognormal(),
    "heat3d_255_N64_lognormal": lambda: heat3d_lognormal(n=255, N=64, seed=1005, contrast=1e3),
}
