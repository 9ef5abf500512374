"""Seeded synthetic inputs for the fractional Allen-Cahn solves.

This module only draws numbers and lays them out; it holds none of the method's arithmetic,
so both the GPU path's tests and the CPU oracle's tests take their inputs from here.

Arrays are float64, C-order, with axis 1 (the paper's x^(1)) fastest: shape (N2, N1) in 2D
and (N3, N2, N1) in 3D. Every generator takes an explicit seed for numpy's default_rng.
"""

from dataclasses import dataclass, field
import math

import numpy as np


@dataclass
class Instance:
    """One solve: grid sizes per axis (axis 1 first), fractional orders per axis, the
    interface parameter eps, time step tau, mesh widths per axis and a step count."""
    ns: tuple
    alphas: tuple
    eps: float
    tau: float
    hs: tuple
    steps: int
    u0: np.ndarray = field(repr=False, default=None)

    @property
    def dims(self):
        return len(self.ns)

    @property
    def points(self):
        return int(np.prod(self.ns))

    @property
    def shape(self):
        return tuple(reversed(self.ns))


def mesh_widths(ns, a=-1.0, b=1.0):
    """h_l = (b - a)/(N_l + 1) for N_l interior nodes (m_l = N_l + 1 intervals)."""
    return tuple((b - a) / (n + 1) for n in ns)


def uniform_field(shape, lo, hi, seed):
    """i.i.d. uniform values in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape)


def _gaussian_taps(sigma):
    r = int(math.ceil(4 * sigma))
    x = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-0.5 * (x / sigma) ** 2)
    return w / w.sum()


def smoothed_tanh_field(shape, seed, sigma=8.0, amp=0.9, gain=2.0):
    """Standard normal noise, separably smoothed by a Gaussian of width sigma grid points
    (taps truncated at 4 sigma, zero outside the grid), rescaled to unit standard deviation,
    then amp * tanh(gain * z) clipped to [-amp, amp]."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(size=shape)
    taps = _gaussian_taps(sigma)
    for ax in range(z.ndim):
        z = np.apply_along_axis(lambda v: np.convolve(v, taps, mode="same"), ax, z)
    z = z / z.std()
    return np.clip(amp * np.tanh(gain * z), -amp, amp)


def two_gaussians_2d(n, length=2.0):
    """Initial value of Example 1 (Sec. 5): two Gaussians of weight 1/2 centred at
    (2/3, 2/3) and (4/3, 4/3) with exponent -100 on (0, 2)^2, sampled at the interior nodes."""
    h = length / (n + 1)
    x = h * np.arange(1, n + 1)
    x1 = x[None, :]
    x2 = x[:, None]
    return (0.5 * np.exp(-100.0 * ((x1 - 2 / 3) ** 2 + (x2 - 2 / 3) ** 2))
            + 0.5 * np.exp(-100.0 * ((x1 - 4 / 3) ** 2 + (x2 - 4 / 3) ** 2)))


def two_gaussians_3d(n, length=1.0):
    """Initial value of Example 2 (Sec. 5): two Gaussians of weight 1/2 centred at
    (3/8, 3/8, 3/8) and (5/8, 5/8, 5/8) with exponent -500 on (0, 1)^3."""
    h = length / (n + 1)
    x = h * np.arange(1, n + 1)
    x1 = x[None, None, :]
    x2 = x[None, :, None]
    x3 = x[:, None, None]
    c1, c2 = 3 / 8, 5 / 8
    return (0.5 * np.exp(-500.0 * ((x1 - c1) ** 2 + (x2 - c1) ** 2 + (x3 - c1) ** 2))
            + 0.5 * np.exp(-500.0 * ((x1 - c2) ** 2 + (x2 - c2) ** 2 + (x3 - c2) ** 2)))


# ------------------------------------------------------------------ benchmark workloads
def plain_2d_63(steps=100):
    """2D plain method: [-1,1]^2, N=63, alpha=(1.5,1.5), eps=0.1, tau=0.01, 100 steps,
    u0 i.i.d. uniform in [-0.9, 0.9] (seed 1)."""
    ns = (63, 63)
    inst = Instance(ns, (1.5, 1.5), 0.1, 0.01, mesh_widths(ns), steps)
    inst.u0 = uniform_field(inst.shape, -0.9, 0.9, seed=1)
    return inst


def large_2d_1023(steps=1000):
    """2D single large instance: [-1,1]^2, N=1023, alpha=(1.3,1.7), eps=0.05, tau=1e-3,
    1000 steps, u0 = clipped 0.9 tanh of a smoothed seeded normal field (seed 2)."""
    ns = (1023, 1023)
    inst = Instance(ns, (1.3, 1.7), 0.05, 1e-3, mesh_widths(ns), steps)
    inst.u0 = smoothed_tanh_field(inst.shape, seed=2)
    return inst


def large_3d_255(steps=200, n=255):
    """3D single instance: [-1,1]^3, N=255, alpha=(1.2,1.5,1.8), eps=0.08, tau=5e-3,
    200 steps, u0 i.i.d. uniform in [-0.5, 0.5] (seed 3)."""
    ns = (n, n, n)
    inst = Instance(ns, (1.2, 1.5, 1.8), 0.08, 5e-3, mesh_widths(ns), steps)
    inst.u0 = uniform_field(inst.shape, -0.5, 0.5, seed=3)
    return inst


def subsample_3d_63(big):
    """The 63^3 companion of the 255^3 instance: h = 2/64 is every 4th node of h = 2/256,
    interior index i -> 4 i; same alpha, eps, tau and steps, u0 sampled at those nodes."""
    ns = (63, 63, 63)
    inst = Instance(ns, big.alphas, big.eps, big.tau, mesh_widths(ns), big.steps)
    inst.u0 = np.ascontiguousarray(big.u0[3::4, 3::4, 3::4])
    return inst


BATCH_SIZES = (63, 127, 255, 511, 1023)


def batched_2d(count=64, steps=500, seed=4, sizes=BATCH_SIZES):
    """Independent 2D instances: n drawn from `sizes` (one n for both axes), alpha per axis
    uniform(1.1, 1.9), eps uniform(0.02, 0.2), tau uniform(1e-3, 1e-2), u0 uniform in
    [-0.9, 0.9], all from one seeded generator."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(sizes))
        a = (float(rng.uniform(1.1, 1.9)), float(rng.uniform(1.1, 1.9)))
        eps = float(rng.uniform(0.02, 0.2))
        tau = float(rng.uniform(1e-3, 1e-2))
        ns = (n, n)
        inst = Instance(ns, a, eps, tau, mesh_widths(ns), steps)
        inst.u0 = rng.uniform(-0.9, 0.9, size=inst.shape)
        out.append(inst)
    return out


@dataclass
class Request:
    """A served solve: arrival time (s), the instance, and its arithmetic type."""
    rid: int
    arrival: float
    inst: Instance
    dtype: str


def served_stream(count=2000, rate=200.0, seed=5, n2=(63, 1023), n3=(31, 255),
                  steps=(50, 2000), materialize=True):
    """Poisson arrivals (exponential gaps of mean 1/rate) of 2D and 3D solves, 2D:3D and
    FP64:FP32 each 1:1 by Bernoulli draws; n uniform on the integer range for its dimension;
    alpha per axis uniform(1.1, 1.9), eps uniform(0.02, 0.2), tau uniform(1e-3, 1e-2),
    steps uniform on the integer range, u0 uniform in [-0.9, 0.9]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += float(rng.exponential(1.0 / rate))
        d = 3 if rng.random() < 0.5 else 2
        dt = "f32" if rng.random() < 0.5 else "f64"
        lo, hi = (n3 if d == 3 else n2)
        n = int(rng.integers(lo, hi + 1))
        ns = (n,) * d
        alphas = tuple(float(rng.uniform(1.1, 1.9)) for _ in range(d))
        eps = float(rng.uniform(0.02, 0.2))
        tau = float(rng.uniform(1e-3, 1e-2))
        st = int(rng.integers(steps[0], steps[1] + 1))
        useed = int(rng.integers(0, 2 ** 31 - 1))
        inst = Instance(ns, alphas, eps, tau, mesh_widths(ns), st)
        if materialize:
            inst.u0 = uniform_field(inst.shape, -0.9, 0.9, useed)
        else:
            inst.u0 = None
            inst.seed = useed
        out.append(Request(rid, t, inst, dt))
    return out


def example3(dims, alphas, seed, steps=None):
    """Sec. 5, Example 3 (phase separation and coarsening): (0, 1)^d, eps = 0.01, tau = 0.1,
    u0 uniform in [-0.9, 0.9]; 255^2 nodes in 2D (t to 100), 127^3 in 3D (t to 200)."""
    n = 255 if dims == 2 else 127
    ns = (n,) * dims
    steps = steps if steps is not None else (1000 if dims == 2 else 2000)
    inst = Instance(ns, tuple(alphas), 0.01, 0.1, tuple(1.0 / (n + 1) for _ in ns), steps)
    inst.u0 = uniform_field(tuple(reversed(ns)), -0.9, 0.9, seed)
    return inst


def example4(dims, alphas, seed, steps):
    """Sec. 5, Example 4 (the discrete maximum principle): Example 3's meshes with eps = 0.1,
    tau = 0.01 and u0 = 0.95 rand + 0.05 (rand uniform in (0, 1))."""
    n = 255 if dims == 2 else 127
    ns = (n,) * dims
    inst = Instance(ns, tuple(alphas), 0.1, 0.01, tuple(1.0 / (n + 1) for _ in ns), steps)
    inst.u0 = 0.95 * uniform_field(tuple(reversed(ns)), 0.0, 1.0, seed) + 0.05
    return inst
