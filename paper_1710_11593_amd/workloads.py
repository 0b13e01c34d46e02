"""Seeded synthetic workloads shaped like the paper's experiments.

This module generates inputs only: grids, manufactured sources and random
smooth source modes.  It holds none of the solver's arithmetic (no weights,
no time stepping) and is shared, as data, by the oracle-based tests and the
HIP path.  All arrays are float64, time-major [N][M] (row n-1 is t_n, column
i-1 is x_i), with h = (x1-x0)/(M+1), x_i = x0 + i h, tau = T/N.

Source sampling follows the schemes: f(x_i, t_n) for 0<gamma<1 (Scheme 4,
eq. e19) and f(x_i, t_{n-1/2}) for 1<gamma<2 (eq. e16/e17).

Recipes (domain [0,1], T = 1):
  diffusion_manufactured  u = t^2 sin(pi x): f = (2 t^(2-g)/Gamma(3-g) + pi^2 t^2) sin(pi x)
  wave_manufactured       u = (t^2+1) sin(pi x), u0 = sin(pi x), phi = 0:
                          f = (2 t^(2-g)/Gamma(3-g) + pi^2 (t^2+1)) sin(pi x)
  random modes            sum_j a_j t^(p_j) sin(j pi x), a_j ~ N(0,1), p_j ~ U(1,3)
                          (draw order: all a, then all p)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def regime(gamma: float) -> str:
    if 0.0 < gamma < 1.0:
        return "diffusion"
    if 1.0 < gamma < 2.0:
        return "wave"
    raise ValueError("gamma must lie in (0,1) or (1,2), got %r" % gamma)


def grid(M: int, N: int, T: float = 1.0, x0: float = 0.0, x1: float = 1.0):
    h = (x1 - x0) / (M + 1)
    tau = T / N
    x = x0 + h * np.arange(1, M + 1)
    t = tau * np.arange(1, N + 1)
    return x, t, h, tau


def sample_times(gamma: float, N: int, T: float = 1.0) -> np.ndarray:
    """Times at which the source is sampled: t_n, or t_{n-1/2} for 1<gamma<2."""
    tau = T / N
    n = np.arange(1, N + 1, dtype=np.float64)
    return tau * (n - 0.5) if regime(gamma) == "wave" else tau * n


def sine(M: int, j: int, x0: float = 0.0, x1: float = 1.0) -> np.ndarray:
    x, _, _, _ = grid(M, 1, 1.0, x0, x1)
    return np.sin(j * math.pi * (x - x0) / (x1 - x0))


def manufactured_source(gamma: float, M: int, N: int, T: float = 1.0):
    """(f, u0, phi, exact) for the manufactured solutions named above."""
    x, t, _, _ = grid(M, N, T)
    ts = sample_times(gamma, N, T)
    s1 = np.sin(math.pi * x)
    c = 2.0 / math.gamma(3.0 - gamma)
    if regime(gamma) == "diffusion":
        g = c * ts ** (2.0 - gamma) + math.pi ** 2 * ts ** 2
        u0 = np.zeros(M)
        exact = np.outer(t ** 2, s1)
    else:
        g = c * ts ** (2.0 - gamma) + math.pi ** 2 * (ts ** 2 + 1.0)
        u0 = s1.copy()
        exact = np.outer(t ** 2 + 1.0, s1)
    f = np.outer(g, s1)
    return f, u0, np.zeros(M), exact


def random_modes(rng: np.random.Generator, nmodes: int):
    a = rng.standard_normal(nmodes)
    p = rng.uniform(1.0, 3.0, nmodes)
    return a, p


def mode_source(gamma, M, N, amps, pows, js, T=1.0):
    """sum_k amps[k] t^pows[k] sin(js[k] pi x) sampled on the scheme's times."""
    ts = sample_times(gamma, N, T)
    x, _, _, _ = grid(M, N, T)
    f = np.zeros((N, M))
    for a, p, j in zip(amps, pows, js):
        f += np.outer(a * ts ** p, np.sin(j * math.pi * x))
    return f


@dataclass
class Instance:
    gamma: float
    M: int
    N: int
    T: float = 1.0
    x0: float = 0.0
    x1: float = 1.0
    f: np.ndarray | None = None
    u0: np.ndarray | None = None
    phi: np.ndarray | None = None
    # modal description of the source: f = sum_k g_k(t) sin(j_k pi x) with
    # g_k(t) = amp_k t^pow_k, plus optional manufactured part (mode 1)
    modes: list = field(default_factory=list)   # (j, amp, pow)
    manufactured: bool = False

    @property
    def unknowns(self) -> int:
        return self.M * self.N


def c1() -> Instance:
    """Diffusion, gamma = 0.5, M = 64, N = 256, u = t^2 sin(pi x)."""
    f, u0, phi, _ = manufactured_source(0.5, 64, 256)
    return Instance(0.5, 64, 256, f=f, u0=u0, phi=phi, manufactured=True)


def c2(gamma: float = 0.3, seed: int = 2, M: int = 4096, N: int = 65536, build: bool = True) -> Instance:
    """Diffusion, M = 4096, N = 2^16: manufactured source + 8 seeded modes j = 1..8."""
    rng = np.random.default_rng(seed)
    amps, pows = random_modes(rng, 8)
    modes = [(j, float(a), float(p)) for j, a, p in zip(range(1, 9), amps, pows)]
    inst = Instance(gamma, M, N, modes=modes, manufactured=True)
    if build:
        fill(inst)
    return inst


def c3(M: int = 2048, N: int = 131072, build: bool = True) -> Instance:
    """Diffusion-wave, gamma = 1.5, u = (t^2+1) sin(pi x), u0 = sin(pi x), phi = 0."""
    inst = Instance(1.5, M, N, manufactured=True)
    if build:
        fill(inst)
    return inst


def c4(seed: int = 4, count: int = 256):
    """256 uneven instances; per instance, in draw order: M, N, regime, gamma, 4 modes."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        M = int(round(math.exp(rng.uniform(math.log(64), math.log(2048)))))
        N = 2 ** int(round(rng.uniform(10, 15)))
        wave = rng.uniform() < 0.5
        gamma = float(rng.uniform(1.1, 1.9) if wave else rng.uniform(0.1, 0.9))
        amps, pows = random_modes(rng, 4)
        modes = [(j, float(a), float(p)) for j, a, p in zip(range(1, 5), amps, pows)]
        out.append(Instance(gamma, M, N, modes=modes, manufactured=False))
    return out


def c5(seed: int = 5, M: int = 1024, N: int = 32768, build: bool = True):
    """Differentiation case, gamma = 0.6: (base instance, observation instance).

    The base source is the manufactured t^2 sin(pi x) term; the observation is
    the solution for the base source plus 0.1 xi_k t^(p_k) sin(j_k pi x) on 4
    distinct modes: j_1 = 1 (the base's own mode, so that u - u_obs has a part
    that the base solution's gamma-dependence meets and dL/dgamma is not zero
    by orthogonality) and j_2..j_4 drawn from 2..32.
    """
    rng = np.random.default_rng(seed)
    js = [1] + [int(j) for j in rng.choice(np.arange(2, 33), size=3, replace=False)]
    xi = rng.standard_normal(4)
    pows = rng.uniform(1.0, 3.0, 4)
    base = Instance(0.6, M, N, manufactured=True)
    pert = [(int(j), 0.1 * float(a), float(p)) for j, a, p in zip(js, xi, pows)]
    obs = Instance(0.6, M, N, modes=list(pert), manufactured=True)
    if build:
        fill(base)
        fill(obs)
    return base, obs


def fill(inst: Instance) -> Instance:
    """Materialise f, u0, phi for an instance from its modal description."""
    M, N, g = inst.M, inst.N, inst.gamma
    f = np.zeros((N, M))
    u0 = np.zeros(M)
    phi = np.zeros(M)
    if inst.manufactured:
        fm, u0, phi, _ = manufactured_source(g, M, N, inst.T)
        f += fm
    if inst.modes:
        js = [m[0] for m in inst.modes]
        f += mode_source(g, M, N, [m[1] for m in inst.modes], [m[2] for m in inst.modes], js, inst.T)
    inst.f, inst.u0, inst.phi = f, u0, phi
    return inst


def modal_time_series(inst: Instance):
    """Per sine mode j: (g^n sampled on the scheme's times, u0 coefficient, phi coefficient).

    Exactly the data that make f = sum_j g_j(t_n) sin(j pi x_i); used to pin
    full-size solutions through the single-mode scalar recurrence.
    """
    ts = sample_times(inst.gamma, inst.N, inst.T)
    out = {}
    if inst.manufactured:
        c = 2.0 / math.gamma(3.0 - inst.gamma)
        if regime(inst.gamma) == "diffusion":
            out[1] = [c * ts ** (2.0 - inst.gamma) + math.pi ** 2 * ts ** 2, 0.0, 0.0]
        else:
            out[1] = [c * ts ** (2.0 - inst.gamma) + math.pi ** 2 * (ts ** 2 + 1.0), 1.0, 0.0]
    for j, a, p in inst.modes:
        series = a * ts ** p
        if j in out:
            out[j][0] = out[j][0] + series
        else:
            out[j] = [series, 0.0, 0.0]
    return out
