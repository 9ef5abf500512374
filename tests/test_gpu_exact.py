"""The one-level scheme with the exact exponential (eq. (strang)) on the GPU, SFAC_METHOD_EXACT.

This is the scheme the paper sets the two-level method against in Tables 2 and 4: one step is
J^Q_{tau/2} e^{tau A} J^Q_{tau/2}, and e^{tau A} (A the Kronecker sum of the axes' B) is the
product of the per-axis factors e^{tau B_l}, each one dense FP64 product along its axis.

* parity with the oracle's strang_solve, element by element, at sizes with several 64-wide
  product tiles and ragged tails, in 1D, 2D and 3D;
* bitwise the same with and without graphs and across split calls;
* the paper's printed Strang columns: Table 2 (2D, 255^2) and every row of Table 4 (3D, 63^3);
* the per-step max|u| record and the energy work on such a plan as on the two-level one.
"""
import json
import os

import numpy as np
import pytest
from conftest import progress

from oracle import sfac_oracle as O
from paper_2209_08437_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FP64_TOL = 1e-12     # relative to max|u|, as for the two-level FP64 path


def _say(msg):
    progress(msg)   # past the output capture: long tests show they are alive


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _run(u0, ns, alphas, eps, hs, tau, steps, splits=None, use_graph=True):
    import torch
    from paper_2209_08437_amd import sfac
    u = torch.tensor(np.ascontiguousarray(u0), dtype=torch.float64, device="cuda")
    with sfac.Plan(ns, alphas, eps, tau, hs, "f64", method="exact", use_graph=use_graph) as p:
        for a in range(len(ns)):
            assert p.method(a + 1) == ("exact", ns[a])
        for k in (splits or [steps]):
            p.step(u, k)
        flags, vmax = p.flags()
    torch.cuda.synchronize()
    return u.cpu().numpy(), flags, vmax


@pytest.mark.parametrize("ns,alphas,eps,tau", [
    ((200,), (1.7,), 0.1, 0.01),
    ((63, 130), (1.3, 1.8), 0.1, 0.01),          # 1 and 3 tiles of 64, ragged
    ((17, 9, 33), (1.3, 1.6, 1.9), 0.3, 0.02),   # every axis below or just over one tile
    ((70, 5, 66), (1.2, 1.5, 1.1), 0.05, 0.05),
], ids=lambda v: str(v))
def test_exact_parity_with_oracle(sfac_lib, ns, alphas, eps, tau):
    hs = W.mesh_widths(ns)
    u0 = W.uniform_field(tuple(reversed(ns)), -0.95, 0.95, seed=7 + len(ns))
    steps = 12
    ref = O.strang_solve(u0, ns, alphas, eps, hs, tau, steps)
    _say(f"case exact {ns} {alphas}")
    got, flags, vmax = _run(u0, ns, alphas, eps, hs, tau, steps)
    rel = np.abs(got - ref).max() / np.abs(ref).max()
    _say(f"  max rel diff {rel:.2e}, flags {flags}, max|u| {vmax:.6f}")
    assert rel <= FP64_TOL
    assert flags == 0 and vmax >= np.abs(got).max()
    # split calls and plain launches give the same bits
    split, _, _ = _run(u0, ns, alphas, eps, hs, tau, steps, splits=[5, 0, 7])
    plain, _, _ = _run(u0, ns, alphas, eps, hs, tau, steps, use_graph=False)
    assert np.array_equal(split, got) and np.array_equal(plain, got)


@pytest.mark.parametrize("which,steps", [("large_2d_1023", 20), ("large_3d_255", 3)])
def test_exact_parity_full_size(sfac_lib, which, steps):
    """The benchmark workloads at full size (1023^2 and 255^3 FP64), every element against the
    oracle's one-level solve: the products then span 32 and 8 tiles of 32 per axis, with the
    ragged last tile, and the 3D strided axes run as batches of 255."""
    inst = getattr(W, which)()
    ref = O.strang_solve(inst.u0, inst.ns, inst.alphas, inst.eps, inst.hs, inst.tau, steps)
    _say(f"case exact full size {which}, {steps} steps")
    got, flags, _ = _run(inst.u0, inst.ns, inst.alphas, inst.eps, inst.hs, inst.tau, steps)
    rel = np.abs(got - ref).max() / np.abs(ref).max()
    _say(f"  max rel diff {rel:.2e}")
    assert rel <= FP64_TOL and flags == 0


def test_exact_maximum_length(sfac_lib):
    """N = 1024, the longest axis an exact plan takes, on both the contiguous and the strided
    axis (1024 x 3 and 3 x 1024), against the oracle."""
    for ns in ((1024, 3), (3, 1024)):
        hs = W.mesh_widths(ns)
        u0 = W.uniform_field(tuple(reversed(ns)), -0.9, 0.9, seed=sum(ns))
        ref = O.strang_solve(u0, ns, (1.9, 1.2), 0.1, hs, 0.01, 5)
        got, flags, _ = _run(u0, ns, (1.9, 1.2), 0.1, hs, 0.01, 5)
        _say(f"case exact maximum length {ns}: {np.abs(got - ref).max() / np.abs(ref).max():.2e}")
        assert flags == 0 and np.abs(got - ref).max() <= FP64_TOL * np.abs(ref).max()


def test_exact_eps0_is_the_nonlinear_flow(sfac_lib):
    """eps = 0: B = 0, e^{tau B} = I, and a step is the closed-form ODE flow over tau."""
    ns = (65, 40)
    u0 = W.uniform_field(tuple(reversed(ns)), -0.9, 0.9, seed=3)
    tau, steps = 0.05, 10
    got, flags, _ = _run(u0, ns, (1.5, 1.5), 0.0, W.mesh_widths(ns), tau, steps)
    t = tau * steps
    ref = u0 / np.sqrt(u0 ** 2 + (1 - u0 ** 2) * np.exp(-2 * t))
    assert np.abs(got - ref).max() <= 1e-13
    assert flags == 0


def test_exact_alpha2_matches_sine_transform(sfac_lib):
    """alpha = 2: B is eps^2/h^2 tridiag(1, -2, 1), whose eigenvectors are the DST-I sine modes
    with eigenvalues -(4 eps^2 / h^2) sin^2(j pi / (2 (N + 1))). The step built from that closed
    form and the exact flow of the nonlinear half-steps, written here independently of the
    oracle, against the GPU's exact scheme."""
    ns, eps, tau, steps = (40, 70), 0.2, 0.05, 5
    hs = W.mesh_widths(ns)
    u0 = W.uniform_field(tuple(reversed(ns)), -0.9, 0.9, seed=31)

    def sine_exponential(n, h):
        j = np.arange(1, n + 1)
        V = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(j, j) * np.pi / (n + 1))
        lam = -(4 * eps ** 2 / h ** 2) * np.sin(j * np.pi / (2 * (n + 1))) ** 2
        return (V * np.exp(tau * lam)[None, :]) @ V.T

    def half(u):     # the Bernoulli flow v' = v - v^3 over tau / 2
        return u / np.sqrt(u * u + (1 - u * u) * np.exp(-tau))

    P1, P2 = sine_exponential(ns[0], hs[0]), sine_exponential(ns[1], hs[1])
    ref = np.array(u0)
    for _ in range(steps):
        ref = half(P2 @ half(ref) @ P1.T)     # axis 1 is the last array dimension
    got, flags, _ = _run(u0, ns, (2.0, 2.0), eps, hs, tau, steps)
    assert flags == 0
    assert np.abs(got - ref).max() <= FP64_TOL * np.abs(ref).max()


@pytest.mark.parametrize("ns", [(1,), (2,), (2, 2), (1, 2), (2, 1, 2), (2, 2, 2)], ids=lambda s: "x".join(map(str, s)))
def test_two_level_equals_exact_for_axes_of_one_or_two(sfac_lib, ns):
    """With N <= 2 on every axis the skew-circulant part is a multiple of I and commutes with the
    circulant part, so the two-level step is the one-level step exactly: the two GPU paths
    agree to rounding."""
    import torch
    from paper_2209_08437_amd import sfac
    alphas = tuple(1.2 + 0.3 * a for a in range(len(ns)))
    hs = W.mesh_widths(ns)
    u0 = W.uniform_field(tuple(reversed(ns)), -0.95, 0.95, seed=len(ns) + sum(ns))
    exact, _, _ = _run(u0, ns, alphas, 0.3, hs, 0.05, 30)
    u = torch.tensor(u0, device="cuda")
    with sfac.Plan(ns, alphas, 0.3, 0.05, hs, "f64") as p:
        p.step(u, 30)
    two = u.cpu().numpy()
    # the oracle's own two schemes differ by up to 1.5e-14 here after 30 steps (rounding only)
    assert np.abs(two - exact).max() <= 1e-13 * np.abs(exact).max()


def test_table2_strang_column(sfac_lib):
    """Sec. 5, Example 1, Table 2 (Strang column): ||u(h, tau) - u(h, tau/2)||_inf on 255 x 255
    interior nodes, T = 1, for all four alpha pairs and tau = 1/100, 1/200."""
    g = _golden("table2_example1_temporal.json")
    n, L, eps, T = g["n"], g["domain_length"], g["eps"], g["T"]
    h = L / (n + 1)
    u0 = W.two_gaussians_2d(n, L)
    cache = {}

    def run(alpha, tau):
        key = (tuple(alpha), tau)
        if key not in cache:
            u, flags, _ = _run(u0, (n, n), alpha, eps, (h, h), tau, int(round(T / tau)))
            assert flags == 0
            cache[key] = u
        return cache[key]

    for row in g["rows"]:
        a, tau = row["alpha"], row["tau"]
        e = np.abs(run(a, tau) - run(a, tau / 2)).max()
        _say(f"case table 2 Strang alpha {a} tau {tau}: {e:.5e} (printed {row['strang']:.5e})")
        assert abs(e - row["strang"]) <= 5e-4 * row["strang"], (a, tau, e, row["strang"])


def test_table4_strang_column(sfac_lib):
    """Sec. 5, Example 2, Table 4 (Strang column), every printed row: the same temporal error on
    63^3 interior nodes of (0, 1)^3, T = 1, tau = 1/20 .. 1/320 for the four alpha sets. The
    solve times of this scheme and of the two-level one are printed beside (the paper's table
    has CPU times of its own implementations; these are one MI355X's)."""
    import time
    import torch
    g = _golden("table4_example2_strang.json")
    n, L, eps = g["n"], g["domain_length"], g["eps"]
    h = L / (n + 1)
    u0 = W.two_gaussians_3d(n, L)
    cache = {}

    def run(alpha, tau_inv):
        key = (tuple(alpha), tau_inv)
        if key not in cache:
            torch.cuda.synchronize()
            t = time.perf_counter()
            u, flags, _ = _run(u0, (n,) * 3, alpha, eps, (h,) * 3, 1.0 / tau_inv, tau_inv)
            assert flags == 0
            cache[key] = (u, time.perf_counter() - t)
        return cache[key]

    for row in g["rows_all"]:
        a, ti = row["alpha"], row["tau_inv"]
        (u1, t1), (u2, _) = run(a, ti), run(a, 2 * ti)
        e = np.abs(u1 - u2).max()
        _say(f"case table 4 Strang alpha {a} tau 1/{ti}: {e:.5e} (printed {row['strang']:.5e}), solve {t1 * 1e3:.1f} ms")
        assert abs(e - row["strang"]) <= 5e-4 * row["strang"], (a, ti, e, row["strang"])


def test_exact_trace_and_energy(sfac_lib):
    """The per-step max|u| record and the discrete energy on a plan of the exact exponential,
    against the oracle's one-level states."""
    import torch
    from paper_2209_08437_amd import sfac
    ns, alphas, eps, tau = (63, 130), (1.4, 1.7), 0.1, 0.02
    hs = W.mesh_widths(ns)
    u0 = W.uniform_field(tuple(reversed(ns)), -0.95, 0.95, seed=19)
    ops = O.axis_operators(ns, alphas, eps, hs, tau)
    steps = 40
    maxes, u = [], np.array(u0)
    for _ in range(steps):
        u = O.strang_step(u, ops, tau)
        maxes.append(np.abs(u).max())
    e_ref = O.discrete_energy(u, ops, hs)
    d = torch.tensor(u0, device="cuda")
    with sfac.Plan(ns, alphas, eps, tau, hs, "f64", method="exact") as p:
        p.trace(steps)
        p.step(d, 25)
        p.step(d, 15)
        rec, n = p.read_trace()
        energy = p.energy(d)
        _, vmax = p.flags()
    assert n == steps
    assert np.abs(rec - np.array(maxes)).max() <= FP64_TOL
    assert rec.max() == vmax
    # the state differs from the oracle's by the FP64 parity bound; the energy is smooth in it
    assert abs(energy - e_ref) <= 1e-11 * abs(e_ref)


def test_exact_plan_product_timing_and_groups(sfac_lib):
    """sfac_plan_time_passes on an exact plan times each axis' dense product and advances the
    state exactly as sfac_step does; groups refuse exact plans."""
    import torch
    from paper_2209_08437_amd import sfac
    ns = (31, 47, 9)
    hs = W.mesh_widths(ns)
    u0 = W.uniform_field(tuple(reversed(ns)), -0.9, 0.9, seed=5)
    args = (ns, (1.5, 1.3, 1.8), 0.1, 0.01, hs, "f64")
    a = torch.tensor(u0, device="cuda")
    b = torch.tensor(u0, device="cuda")
    g = sfac.Group()
    try:
        with sfac.Plan(*args, method="exact") as p:
            p.trace(10)
            ms = p.time_passes(a, 4)
            assert len(ms) == 3 and all(t > 0 for t in ms)
            assert p.read_trace()[1] == 0          # timing is not part of the per-step record
            p.step(b, 4)
            with pytest.raises(sfac.SfacError, match="exact exponential"):
                g.step([p], [b], [1])
    finally:
        g.close()
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_exact_flags_report_nonfinite_and_above_one(sfac_lib):
    """The closing half-step of the exact scheme keeps the sticky status as the two-level passes
    do: a NaN in the state and |u| above 1 (|u0| > 1 leaves Theorem 1's premise) are reported."""
    import torch
    from paper_2209_08437_amd import sfac
    ns = (16, 20, 3)
    hs = W.mesh_widths(ns)
    u0 = W.uniform_field(tuple(reversed(ns)), -0.9, 0.9, seed=1)
    with sfac.Plan(ns, (1.5, 1.5, 1.2), 0.1, 0.01, hs, "f64", method="exact") as p:
        u = torch.tensor(u0, device="cuda")
        p.step(u, 3)
        f, m = p.flags()
        assert f == 0 and 0 < m <= 1
        u[1, 3, 4] = float("nan")
        p.step(u, 1)
        f, _ = p.flags()
        assert f & sfac.FLAG_NONFINITE
        p.reset_flags()
        u = torch.tensor(u0 * 1.5, device="cuda")
        p.step(u, 1)
        f, m = p.flags()
        assert f & sfac.FLAG_ABOVE_ONE and m > 1
