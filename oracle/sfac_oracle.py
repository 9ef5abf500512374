"""Plain FP64 CPU oracle for the two-level Strang splitting of the spatial fractional
Allen-Cahn equation (Cai, Fang, Chen, Sun, arXiv 2209.08437).

TEST INFRASTRUCTURE ONLY. This module exists to check the GPU library; it is not part of
the product. Only the test suite, the package's smoke check and the benchmark's CPU
baseline leg may import it. It shares no code, table or constant with the GPU path.

What it computes, in the paper's order and notation (Sec. 2):

* eq. (g_coe) and eq. (omega_coe): the weights g_k and omega_k;
* eq. (B) with the matrix D_alpha of Sec. 2.1: the symmetric Toeplitz matrix
  B_alpha = kappa (D_alpha + D_alpha^T), kappa = -eps^2 / (2 h^alpha cos(alpha pi / 2));
* eqs. (C) and (S): the circulant C_alpha and skew-circulant S_alpha with B = C + S;
* Remark 1: their spectra through the Fourier matrix F and the diagonal Psi, and from them
  the dense matrices exp(t C) = F* diag(e^{t lambda}) F and exp(t S) = Psi* F* diag(e^{t mu}) F Psi;
* eq. (nonlinear_operator): the closed-form nonlinear flow J^Q_t;
* eq. (hatv) and eq. (finalstrang): one step of the two-level scheme,
  J^Q_{tau/2} e^{tau/2 C_a} e^{tau S_a} e^{tau/2 C_a} J^Q_{tau/2}, where C_a and S_a are the
  Kronecker sums of eq. (2DA) / (3DA) form, so each exponential is the product of the
  per-axis exponentials (all axes' C factors, then all S factors, then all C factors);
* the same step with the per-axis factors multiplied out once (P_l = e^{tau/2 C_l} e^{tau S_l}
  e^{tau/2 C_l}, one dense product per axis, axes in reverse order): a second FP64 evaluation
  order of eq. (finalstrang), used to measure the rounding floor of long runs;
* the same step with every factor applied through Remark 1's diagonalisation by a library FFT
  (a third FP64 evaluation order, for the same measurement), and that evaluation carried out in
  extended precision (numpy's longdouble, every table included): the reference long FP64 runs
  are measured against, since the FP64 orders above differ from it by about as much as they
  differ from each other;
* eq. (strang) with eq. (linear_operator): the one-level scheme with the exact exponential
  e^{tau A}, used only to reproduce the paper's "Strang splitting" table columns;
* Sec. 5, Example 5: the discrete free energy prod(h) (1/4 |u^2 - 1|^2 - 1/2 u^T A u).

Every linear factor is a dense N x N matrix applied by a dense product along one axis of
the state (the FFT evaluation order above aside, which exists only to measure rounding); there
is no blocking or fusion. Arrays are C-order with axis 1 (the paper's
x^(1), index i) fastest, i.e. shape (N2, N1) in 2D and (N3, N2, N1) in 3D, as the state
vector ordering of Sec. 2.1 prescribes.

Index convention: the paper's m is the number of mesh intervals; the unknowns are the
N = m - 1 interior nodes, and every matrix here is N x N.
"""

import numpy as np

__all__ = [
    "g_coefficients", "omega_weights", "riesz_factor", "matrix_D", "matrix_B",
    "toeplitz_column", "circulant_skew_split", "fourier_matrix", "skew_diagonal",
    "circulant_spectrum", "skew_spectrum", "exp_circulant", "exp_skew",
    "exp_symmetric", "nonlinear_flow", "AxisOperators", "axis_operators",
    "apply_along_axis", "two_level_step", "two_level_solve", "composed_operators",
    "two_level_solve_composed", "apply_exp_circulant_fft", "apply_exp_skew_fft",
    "two_level_solve_fft", "extended_solve", "rounding_spread", "strang_step",
    "strang_solve", "discrete_energy",
]


# ----------------------------------------------------------------------------- weights
def _pi(dtype):
    """pi in the precision of `dtype` (numpy's np.pi is a float64 constant)."""
    return np.arccos(dtype(-1))


def g_coefficients(alpha, count, dtype=np.float64):
    """g_0 .. g_{count-1} by the recursion of eq. (g_coe), Sec. 2.1:
    g_0 = 1, g_{k+1} = (1 - (alpha + 1)/(k + 1)) g_k. `dtype` is the arithmetic (float64, or
    numpy's longdouble for the extended-precision reference)."""
    alpha = dtype(alpha)
    g = np.empty(count, dtype=dtype)
    g[0] = 1.0
    for k in range(count - 1):
        g[k + 1] = (1.0 - (alpha + 1.0) / (k + 1.0)) * g[k]
    return g


def omega_weights(alpha, count, dtype=np.float64):
    """omega_0 .. omega_{count-1} of eq. (omega_coe), Sec. 2.1:
    omega_0 = (alpha/2) g_0, omega_{k+1} = (alpha/2) g_{k+1} + ((2 - alpha)/2) g_k."""
    g = g_coefficients(alpha, count, dtype)
    alpha = dtype(alpha)
    w = np.empty(count, dtype=dtype)
    w[0] = 0.5 * alpha * g[0]
    for k in range(count - 1):
        w[k + 1] = 0.5 * alpha * g[k + 1] + 0.5 * (2.0 - alpha) * g[k]
    return w


def riesz_factor(alpha, eps, h, dtype=np.float64):
    """The scalar -eps^2 / (2 h^alpha cos(alpha pi / 2)) that multiplies D + D^T in eq. (B)
    (it is the factor of both sums in eq. (disFAC))."""
    alpha, eps, h = dtype(alpha), dtype(eps), dtype(h)
    return -(eps * eps) / (2 * h ** alpha * np.cos(alpha * _pi(dtype) / 2))


# ---------------------------------------------------------------------- Toeplitz matrix
def matrix_D(alpha, N, dtype=np.float64):
    """D_alpha of Sec. 2.1 as an N x N dense matrix (N = m - 1 interior nodes):
    entry (i, j) is omega_{i - j + 1} when i - j + 1 >= 0 and zero otherwise, i.e.
    omega_1 on the diagonal, omega_0 on the superdiagonal, omega_2, omega_3, ... below."""
    w = omega_weights(alpha, N + 1, dtype)
    i = np.arange(N)[:, None]
    j = np.arange(N)[None, :]
    k = i - j + 1
    D = np.where(k >= 0, w[np.clip(k, 0, N)], dtype(0))
    return D


def matrix_B(alpha, eps, h, N, dtype=np.float64):
    """B_alpha = kappa (D_alpha + D_alpha^T), eq. (B) of Sec. 2.1 (symmetric Toeplitz)."""
    D = matrix_D(alpha, N, dtype)
    return riesz_factor(alpha, eps, h, dtype) * (D + D.T)


def toeplitz_column(B):
    """Diagonal values b_k = B[i, j] for k = i - j, k = -(N-1) .. N-1, as a function."""
    N = B.shape[0]

    def b(k):
        if k >= 0:
            return B[k, 0]
        return B[0, -k]

    return b, N


def circulant_skew_split(B):
    """Dense C_alpha and S_alpha of eqs. (C) and (S): the k-th diagonal of C is
    (b_k + b_{k-N})/2 for k > 0, b_0/2 for k = 0, (b_k + b_{k+N})/2 for k < 0; S takes the
    differences instead. (The paper writes k - m + 1 with m - 1 = N.)"""
    b, N = toeplitz_column(B)
    cdiag = {}
    sdiag = {}
    for k in range(-(N - 1), N):
        if k == 0:
            cdiag[k] = 0.5 * b(0)
            sdiag[k] = 0.5 * b(0)
        elif k > 0:
            cdiag[k] = 0.5 * (b(k) + b(k - N))
            sdiag[k] = 0.5 * (b(k) - b(k - N))
        else:
            cdiag[k] = 0.5 * (b(k) + b(k + N))
            sdiag[k] = 0.5 * (b(k) - b(k + N))
    i = np.arange(N)[:, None]
    j = np.arange(N)[None, :]
    kk = i - j
    cvals = np.array([cdiag[k] for k in range(-(N - 1), N)])
    svals = np.array([sdiag[k] for k in range(-(N - 1), N)])
    C = cvals[kk + (N - 1)]
    S = svals[kk + (N - 1)]
    return C, S


# -------------------------------------------------------------------------- Remark 1
def fourier_matrix(N, dtype=np.float64):
    """The unitary Fourier matrix of Remark 1: F[j, k] = exp(2 pi i j k / N) / sqrt(N).
    The angle is reduced exactly in integers (j k mod N) before the trigonometric call."""
    j = np.arange(N, dtype=np.int64)[:, None]
    k = np.arange(N, dtype=np.int64)[None, :]
    r = (j * k) % N
    ang = 2 * _pi(dtype) * r.astype(dtype) / dtype(N)
    return (np.cos(ang) + 1j * np.sin(ang)) / np.sqrt(dtype(N))


def skew_diagonal(N, dtype=np.float64):
    """Psi = diag(1, e^{-i pi/N}, ..., e^{-i pi (N-1)/N}) of Remark 1, as a vector."""
    k = np.arange(N, dtype=dtype)
    ang = -_pi(dtype) * k / dtype(N)
    return np.cos(ang) + 1j * np.sin(ang)


def circulant_spectrum(C):
    """Eigenvalues of the circulant C by Remark 1: F C e_1 = Lambda_C 1 / sqrt(N), so
    lambda = sqrt(N) F (C e_1). C is symmetric, so lambda is real. Computed in C's precision."""
    N = C.shape[0]
    dt = C.dtype.type
    lam = np.sqrt(dt(N)) * (fourier_matrix(N, dt) @ C[:, 0])
    return lam.real


def skew_spectrum(S):
    """Eigenvalues of the skew-circulant S by Remark 1: F Psi S e_1 = Lambda_S 1 / sqrt(N)."""
    N = S.shape[0]
    dt = S.dtype.type
    mu = np.sqrt(dt(N)) * (fourier_matrix(N, dt) @ (skew_diagonal(N, dt) * S[:, 0]))
    return mu.real


def exp_circulant(C, t):
    """exp(t C) = F* diag(e^{t lambda}) F (Remark 1), a dense real N x N matrix."""
    N = C.shape[0]
    F = fourier_matrix(N)
    lam = circulant_spectrum(C)
    E = F.conj().T @ (np.exp(t * lam)[:, None] * F)
    return E.real


def exp_skew(S, t):
    """exp(t S) = Psi* F* diag(e^{t mu}) F Psi (Remark 1), a dense real N x N matrix."""
    N = S.shape[0]
    F = fourier_matrix(N)
    psi = skew_diagonal(N)
    mu = skew_spectrum(S)
    G = F * psi[None, :]                      # F Psi
    E = G.conj().T @ (np.exp(t * mu)[:, None] * G)
    return E.real


def exp_symmetric(B, t):
    """exp(t B) for a real symmetric B through its eigendecomposition (numpy eigh), used
    for the exact linear flow e^{tau A} of eq. (linear_operator) in the one-level scheme."""
    w, V = np.linalg.eigh(B)
    return (V * np.exp(t * w)[None, :]) @ V.T


# ------------------------------------------------------------------------ nonlinear part
def nonlinear_flow(v, t):
    """J^Q_t of eq. (nonlinear_operator): v / sqrt(v^2 + (1 - v^2) e^{-2t}), the exact flow
    of the Bernoulli equation v' = v - v^3, applied pointwise."""
    v = np.asarray(v)
    if v.dtype != np.longdouble:
        v = v.astype(np.float64)
    t = v.dtype.type(t)
    return v / np.sqrt(v * v + (1 - v * v) * np.exp(-2 * t))


# ---------------------------------------------------------------------- per-axis factors
class AxisOperators:
    """Dense per-axis matrices for one axis: B, C, S and the factors exp(tau/2 C), exp(tau S),
    plus the exact exp(tau B) on request. `dtype` float64, or numpy's longdouble for the
    extended-precision reference (which uses only B, C, S and the spectra: the dense factors
    are formed on first use)."""

    def __init__(self, N, alpha, eps, h, tau, dtype=np.float64):
        self.N, self.alpha, self.eps, self.h, self.tau = N, alpha, eps, h, tau
        self.dtype = dtype
        self.B = matrix_B(alpha, eps, h, N, dtype)
        self.C, self.S = circulant_skew_split(self.B)
        self._EC = self._ES = self._EB = None

    @property
    def EC(self):
        if self._EC is None:
            self._EC = exp_circulant(self.C, 0.5 * self.tau)
        return self._EC

    @property
    def ES(self):
        if self._ES is None:
            self._ES = exp_skew(self.S, self.tau)
        return self._ES

    @property
    def EB(self):
        if self._EB is None:
            self._EB = exp_symmetric(self.B, self.tau)
        return self._EB


def axis_operators(ns, alphas, eps, hs, tau, dtype=np.float64):
    """AxisOperators for axes 1..d (ns, alphas, hs are per-axis sequences, axis 1 first)."""
    return [AxisOperators(int(n), float(a), float(eps), float(h), float(tau), dtype)
            for n, a, h in zip(ns, alphas, hs)]


def apply_along_axis(M, u, axis):
    """Apply the N x N matrix M to every line of u along the paper's axis `axis` (1-based,
    axis 1 = last array dimension), i.e. the Kronecker factor I x .. x M x .. x I."""
    d = u.ndim
    ax = d - axis
    out = np.tensordot(M, u, axes=([1], [ax]))
    return np.moveaxis(out, 0, ax)


def two_level_step(u, ops, tau):
    """One step of eq. (finalstrang): J^Q_{tau/2} (e^{tau/2 C_a} e^{tau S_a} e^{tau/2 C_a}) J^Q_{tau/2}.
    Each Kronecker-sum exponential is applied as the product of its per-axis factors."""
    d = u.ndim
    u = nonlinear_flow(u, 0.5 * tau)
    for ax in range(1, d + 1):
        u = apply_along_axis(ops[ax - 1].EC, u, ax)
    for ax in range(1, d + 1):
        u = apply_along_axis(ops[ax - 1].ES, u, ax)
    for ax in range(1, d + 1):
        u = apply_along_axis(ops[ax - 1].EC, u, ax)
    u = nonlinear_flow(u, 0.5 * tau)
    return u


def two_level_solve(u0, ns, alphas, eps, hs, tau, nsteps, ops=None, observe=None):
    """nsteps steps of the two-level scheme from u0 (shape (N_d, .., N_1)). `observe`, if
    given, is called with (step index, state) after every step."""
    u = np.array(u0, dtype=np.float64, copy=True)
    if ops is None:
        ops = axis_operators(ns, alphas, eps, hs, tau)
    for n in range(nsteps):
        u = two_level_step(u, ops, tau)
        if observe is not None:
            observe(n + 1, u)
    return u


def composed_operators(ops):
    """Per axis the dense product P_l = e^{tau/2 C_l} e^{tau S_l} e^{tau/2 C_l}, formed once. The
    Kronecker-sum exponentials of eq. (finalstrang) factor per axis and factors on different axes
    commute, so the linear part of a step is the product over the axes of these P_l."""
    return [op.EC @ op.ES @ op.EC for op in ops]


def two_level_solve_composed(u0, ns, alphas, eps, hs, tau, nsteps, ops=None, reverse_axes=True, observe=None):
    """The scheme of two_level_solve evaluated in another FP64 order: each step applies the
    composed per-axis operators P_l (one dense product per axis), the last axis first when
    `reverse_axes` is set. Equal to two_level_solve in exact arithmetic; the two differ only by
    rounding, which measures how reproducible an FP64 evaluation of a long run is at all.
    `observe`, if given, is called as observe(step, u) after every step."""
    u = np.array(u0, dtype=np.float64, copy=True)
    if ops is None:
        ops = axis_operators(ns, alphas, eps, hs, tau)
    P = composed_operators(ops)
    d = u.ndim
    order = range(d, 0, -1) if reverse_axes else range(1, d + 1)
    for n in range(nsteps):
        u = nonlinear_flow(u, 0.5 * tau)
        for ax in order:
            u = apply_along_axis(P[ax - 1], u, ax)
        u = nonlinear_flow(u, 0.5 * tau)
        if observe is not None:
            observe(n + 1, u)
    return u


def _fft_module(x):
    """numpy's FFT for float64 data; scipy's (which keeps numpy's longdouble) for the extended
    reference, split over the host's threads."""
    if x.dtype in (np.longdouble, np.clongdouble):
        import os
        import scipy.fft as sfft
        w = os.cpu_count() or 1
        return (lambda a, axis: sfft.fft(a, axis=axis, workers=w)), (lambda a, axis: sfft.ifft(a, axis=axis, workers=w))
    return np.fft.fft, np.fft.ifft


def apply_exp_circulant_fft(x, lam, t, axis):
    """e^{t C} along the paper's axis `axis` through Remark 1 with a library FFT: C = F* Lambda F
    with F = sqrt(N) ifft (the e^{+2 pi i j k / N} / sqrt(N) of Remark 1) and F* = fft / sqrt(N)."""
    ax = x.ndim - axis
    shape = [1] * x.ndim
    shape[ax] = -1
    fft, ifft = _fft_module(x)
    e = np.exp(lam.dtype.type(t) * lam).reshape(shape)
    return fft(e * ifft(x, axis=ax), axis=ax).real


def apply_exp_skew_fft(x, mu, t, axis):
    """e^{t S} along `axis` through Remark 1 with a library FFT: S = Psi* F* Lambda_S F Psi."""
    ax = x.ndim - axis
    N = x.shape[ax]
    shape = [1] * x.ndim
    shape[ax] = -1
    fft, ifft = _fft_module(x)
    psi = skew_diagonal(N, x.dtype.type).reshape(shape)
    e = np.exp(mu.dtype.type(t) * mu).reshape(shape)
    y = ifft(psi * x, axis=ax)
    return (np.conj(psi) * fft(e * y, axis=ax)).real


def two_level_solve_fft(u0, ns, alphas, eps, hs, tau, nsteps, ops=None, dtype=np.float64, observe=None):
    """The scheme of two_level_solve evaluated through Remark 1's diagonalisation with a library
    FFT instead of dense products, in the paper's factor order. In float64 it is a third
    evaluation order (used beside two_level_solve_composed to measure how far FP64 evaluations
    of a long run spread). With dtype=numpy.longdouble every table (g, omega, B, C, S, the
    spectra, Psi) and every operation is carried in extended precision (64-bit significand on
    x86, unit roundoff 2^-64): the reference the FP64 results are measured against, about 2000
    times more precise than any FP64 evaluation. Returns an array of `dtype`. `observe`, if given,
    is called as observe(step, u) after every step."""
    u = np.array(u0, dtype=dtype, copy=True)
    if ops is None or ops[0].dtype != dtype:
        ops = axis_operators(ns, alphas, eps, hs, tau, dtype)
    lams = [circulant_spectrum(op.C) for op in ops]
    mus = [skew_spectrum(op.S) for op in ops]
    d = u.ndim
    half = dtype(tau) / 2
    for n in range(nsteps):
        u = nonlinear_flow(u, half)
        for ax in range(1, d + 1):
            u = apply_exp_circulant_fft(u, lams[ax - 1], half, ax)
        for ax in range(1, d + 1):
            u = apply_exp_skew_fft(u, mus[ax - 1], dtype(tau), ax)
        for ax in range(1, d + 1):
            u = apply_exp_circulant_fft(u, lams[ax - 1], half, ax)
        u = nonlinear_flow(u, half)
        if observe is not None:
            observe(n + 1, u)
    return u


def extended_solve(u0, ns, alphas, eps, hs, tau, nsteps, observe=None):
    """two_level_solve_fft in numpy's longdouble: the extended-precision reference."""
    return two_level_solve_fft(u0, ns, alphas, eps, hs, tau, nsteps, dtype=np.longdouble, observe=observe)


def rounding_spread(u0, ns, alphas, eps, hs, tau, nsteps, ref, ops=None, observe=None):
    """Largest relative max-norm distance of the two other FP64 evaluation orders
    (two_level_solve_composed, two_level_solve_fft) from `ref`, the result of two_level_solve on
    the same input: the spread below which FP64 evaluations of this run are not reproducible.
    `observe` is passed to both solves."""
    if ops is None:
        ops = axis_operators(ns, alphas, eps, hs, tau)
    scale = max(float(np.abs(ref).max()), 1e-300)
    out = 0.0
    for alt in (two_level_solve_composed(u0, ns, alphas, eps, hs, tau, nsteps, ops=ops, observe=observe),
                two_level_solve_fft(u0, ns, alphas, eps, hs, tau, nsteps, ops=ops, observe=observe)):
        out = max(out, float(np.abs(alt - ref).max()) / scale)
    return out


def strang_step(u, ops, tau):
    """One step of eq. (strang): J^Q_{tau/2} e^{tau A} J^Q_{tau/2}, with e^{tau A} the product of
    the exact per-axis exponentials exp(tau B_l) (A is a Kronecker sum, eq. (2DA)/(3DA))."""
    d = u.ndim
    u = nonlinear_flow(u, 0.5 * tau)
    for ax in range(1, d + 1):
        u = apply_along_axis(ops[ax - 1].EB, u, ax)
    return nonlinear_flow(u, 0.5 * tau)


def strang_solve(u0, ns, alphas, eps, hs, tau, nsteps, ops=None):
    u = np.array(u0, dtype=np.float64, copy=True)
    if ops is None:
        ops = axis_operators(ns, alphas, eps, hs, tau)
    for _ in range(nsteps):
        u = strang_step(u, ops, tau)
    return u


def discrete_energy(u, ops, hs):
    """Discrete free energy of Example 5 (Sec. 5): prod(h) (1/4 |u^2 - 1|^2 - 1/2 u^T A u),
    with A the Kronecker sum of the per-axis B matrices."""
    Au = np.zeros_like(u)
    for ax in range(1, u.ndim + 1):
        Au = Au + apply_along_axis(ops[ax - 1].B, u, ax)
    q = u * u - 1.0
    return float(np.prod(hs)) * (0.25 * np.sum(q * q) - 0.5 * np.sum(u * Au))
