// Host-side construction of the per-axis tables (FP64 results from long double arithmetic).
//
// For one axis with N interior nodes, order alpha, mesh width h, parameter eps and step tau:
//   * g_k and omega_k by the recursions of eqs. (g_coe), (omega_coe);
//   * the first column b_k of the symmetric Toeplitz B_alpha = kappa (D + D^T) of eq. (B),
//     kappa = -eps^2 / (2 h^alpha cos(alpha pi / 2)): entry (i, j) of D is omega_{i-j+1}, so
//     b_0 = 2 kappa omega_1, b_1 = kappa (omega_0 + omega_2), b_k = kappa omega_{k+1} (k >= 2);
//   * the first columns of the circulant C and skew-circulant S of eqs. (C), (S):
//     c_0 = s_0 = b_0 / 2, c_k = (b_k + b_{N-k}) / 2, s_k = (b_k - b_{N-k}) / 2;
//   * the spectra of Remark 1 with the forward transform e^{-2 pi i j k / N}:
//     lambda_j = sum_k c_k e^{-2 pi i j k / N},  mu_j = sum_k s_k psi_k e^{-2 pi i j k / N},
//     psi_k = e^{-i pi k / N}; both are real because c and s are symmetric.
// The diagonal method keeps e^{tau/2 lambda_j}/N and e^{tau mu_j}/N (the 1/N of the inverse
// transform folded in). The embedded method turns both exponentials back into their first
// columns (each is a symmetric Toeplitz matrix) and keeps the length-M spectra of those
// columns placed as circular convolution kernels, divided by M.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <string>
#include <vector>

#include "sfac_embed.hpp"
#include "sfac_internal.hpp"

namespace sfac {

namespace {

using ld = long double;
const ld kPi = 3.141592653589793238462643383279502884L;

// cos(pi r / n) for r < 2n, exact integer angle reduction by the caller
std::vector<ld> half_turn_cosines(int n) {
    std::vector<ld> t(2 * (size_t)n);
    for (int r = 0; r < 2 * n; ++r) t[r] = cosl(kPi * (ld)r / (ld)n);
    return t;
}

}  // namespace

int embed_frequency(int p, int log2m, int log2e) {
    const int nst = embed_stages(log2m, log2e);
    int k = 0, mult = 1, rem = log2m;
    for (int s = 0; s < nst; ++s) {
        const int bits = embed_bits(log2m, log2e, s);
        rem -= bits;
        k += (p >> rem) * mult;   // digit of pass s: the block index at that pass
        p &= (1 << rem) - 1;
        mult <<= bits;
    }
    return k;
}

bool diag2_pair(int n, int* a, int* b) {
    // the instantiated (A, B) pairs of the register-resident diagonal kernel (coprime)
    static const int pairs[][2] = {{3, 5}, {5, 7}, {7, 9}, {9, 11}, {11, 13}, {13, 15}, {15, 17}, {5, 9}, {7, 11}};
    for (const auto& pr : pairs)
        if (pr[0] * pr[1] == n) {
            *a = pr[0];
            *b = pr[1];
            return true;
        }
    return false;
}

int embed_length(int n) {
    int m = 2;
    while (m < 2 * n - 1) m <<= 1;
    return m;
}

bool factor_radices(int n, std::vector<int>* radices) {
    radices->clear();
    if (n < 1) return false;
    int e = 0;
    while ((n & 1) == 0) {
        n >>= 1;
        ++e;
    }
    std::vector<int> merged;
    int threes = 0;
    for (int p = 3; n > 1; p += 2) {
        if (p > kMaxPrimeRadix) return false;
        while (n % p == 0) {
            n /= p;
            if (p == 3)
                ++threes;
            else
                merged.push_back(p);
        }
    }
    // pairs of 3s become one radix-9 pass (no more arithmetic than two radix-3 passes)
    for (; threes >= 2; threes -= 2) merged.push_back(9);
    if (threes) merged.push_back(3);
    // powers of two: as few passes as possible, bits spread evenly, each radix <= 16
    if (e > 0) {
        int stages = (e + 3) / 4;
        for (int s = 0; s < stages; ++s) {
            int bits = e / stages + (s < e % stages ? 1 : 0);
            merged.push_back(1 << bits);
        }
    }
    // largest radices first
    for (size_t i = 0; i < merged.size(); ++i)
        for (size_t j = i + 1; j < merged.size(); ++j)
            if (merged[j] > merged[i]) std::swap(merged[i], merged[j]);
    *radices = merged;
    return (int)radices->size() <= kMaxStages;
}

int auto_method(int n, sfac_dtype) {
    // The diagonal method in its register-resident two-step kernel (N = A B for the built pairs)
    // needs no padding and one LDS exchange per transform; the embedded method runs every N in
    // its register-resident kernel; the generic diagonal kernel (every pass through LDS) measured
    // 3-5x slower per pass. So: two-step diagonal where it exists, else embedded while its length
    // fits, else generic diagonal.
    int a = 0, b = 0;
    if (diag2_pair(n, &a, &b)) return SFAC_METHOD_DIAG;
    int m = embed_length(n);
    if (m <= kMaxEmbedLength) return SFAC_METHOD_EMBED;
    std::vector<int> rd;
    if (n <= kMaxDiagLength && factor_radices(n, &rd)) return SFAC_METHOD_DIAG;
    return 0;
}

// eqs. (g_coe), (omega_coe) for omega_0 .. omega_N, then eq. (B): kappa and the first column
// b_0 .. b_{N-1} of the symmetric Toeplitz B (entry (i, j) is b_{|i - j|})
static std::vector<ld> first_column_B(const AxisParams& p) {
    const int N = p.n;
    std::vector<ld> g(N + 2), w(N + 2);
    const ld a = p.alpha;
    g[0] = 1.0L;
    for (int k = 0; k + 1 < N + 2; ++k) g[k + 1] = (1.0L - (a + 1.0L) / (ld)(k + 1)) * g[k];
    w[0] = 0.5L * a * g[0];
    for (int k = 0; k + 1 < N + 2; ++k) w[k + 1] = 0.5L * a * g[k + 1] + 0.5L * (2.0L - a) * g[k];
    const ld kappa = -((ld)p.eps * (ld)p.eps) / (2.0L * powl((ld)p.h, a) * cosl(a * kPi / 2.0L));
    std::vector<ld> b(N);
    b[0] = 2.0L * kappa * w[1];
    if (N >= 2) b[1] = kappa * (w[0] + w[2]);
    for (int k = 2; k < N; ++k) b[k] = kappa * w[k + 1];
    return b;
}

std::string build_exact_exponential(const AxisParams& p, std::vector<double>* P) {
    const int N = p.n;
    if (N < 1) return "N must be >= 1";
    if (N > kMaxExactLength) {
        char msg[128];
        snprintf(msg, sizeof msg, "N = %d exceeds the exact exponential's limit %d", N, kMaxExactLength);
        return msg;
    }
    // B (eq. (B)) as a dense symmetric matrix and its eigendecomposition B = V diag(lambda) V^T,
    // then e^{tau B} = V diag(e^{tau lambda}) V^T. The eigendecomposition is the textbook
    // symmetric one: Householder reduction to tridiagonal form B = Q T Q^T, then implicit QR
    // steps with the Wilkinson shift on T, each a chase of Givens rotations, accumulated into
    // the rows of V^T (rows stay contiguous, so every update walks memory in order).
    const std::vector<ld> b = first_column_B(p);
    std::vector<double> a((size_t)N * N), q((size_t)N * N, 0.0);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) a[(size_t)i * N + j] = (double)b[(size_t)std::abs(i - j)];
    for (int i = 0; i < N; ++i) q[(size_t)i * N + i] = 1.0;
    auto A = [&](int i, int j) -> double& { return a[(size_t)i * N + j]; };
    std::vector<double> d(N), e(N, 0.0), v(N), w(N);
    // Householder: step k maps column k below the diagonal onto a multiple of e_{k+1} with
    // H = I - beta u u^T acting on indices k+1..N-1; the trailing block S becomes H S H, which is
    // S - u z^T - z u^T for y = beta S u and z = y - (beta u^T y / 2) u
    for (int k = 0; k + 2 < N; ++k) {
        const int m = N - k - 1;
        double* x = &A(k, k + 1);
        double nrm2 = 0.0;
        for (int j = 0; j < m; ++j) nrm2 += x[j] * x[j];
        const double nrm = std::sqrt(nrm2);
        if (nrm == 0.0) {
            e[k] = 0.0;
            continue;
        }
        const double alpha = x[0] > 0 ? -nrm : nrm;
        for (int j = 0; j < m; ++j) v[j] = x[j];
        v[0] -= alpha;
        const double beta = 2.0 / (nrm2 - x[0] * alpha - x[0] * alpha + alpha * alpha);
        double uy = 0.0;
        for (int i = 0; i < m; ++i) {
            const double* row = &A(k + 1 + i, k + 1);
            double acc = 0.0;
            for (int j = 0; j < m; ++j) acc += row[j] * v[j];
            w[i] = beta * acc;
            uy += v[i] * w[i];
        }
        const double kk = 0.5 * beta * uy;
        for (int i = 0; i < m; ++i) w[i] -= kk * v[i];
        for (int i = 0; i < m; ++i) {
            double* row = &A(k + 1 + i, k + 1);
            const double vi = v[i], wi = w[i];
            for (int j = 0; j < m; ++j) row[j] -= vi * w[j] + wi * v[j];
        }
        e[k] = alpha;
        // Q = Q H: every row of Q against u
        for (int i = 0; i < N; ++i) {
            double* row = &q[(size_t)i * N + k + 1];
            double acc = 0.0;
            for (int j = 0; j < m; ++j) acc += row[j] * v[j];
            acc *= beta;
            for (int j = 0; j < m; ++j) row[j] -= acc * v[j];
        }
    }
    for (int k = 0; k < N; ++k) d[k] = A(k, k);
    if (N >= 2) e[N - 2] = A(N - 2, N - 1);
    // V^T starts as Q^T; row r of V^T is the eigenvector of d[r] at the end
    std::vector<double> vt((size_t)N * N);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) vt[(size_t)j * N + i] = q[(size_t)i * N + j];
    auto rotate = [&](int k, double c, double s) {   // V <- V R on columns k, k+1
        double* r0 = &vt[(size_t)k * N];
        double* r1 = r0 + N;
        for (int j = 0; j < N; ++j) {
            const double x0 = r0[j], x1 = r1[j];
            r0[j] = c * x0 - s * x1;
            r1[j] = s * x0 + c * x1;
        }
    };
    const double eps = std::numeric_limits<double>::epsilon();
    long long iters = 0;
    for (int hi = N - 1; hi > 0;) {
        // the unreduced block [lo, hi]: off-diagonals below the rounding of their neighbours are zero
        int lo = hi;
        while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
        if (lo == hi) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        if (++iters > 60LL * N) return "the symmetric QR iteration did not converge";
        // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block nearer to d[hi]
        const double dd = 0.5 * (d[hi - 1] - d[hi]);
        const double eh = e[hi - 1];
        const double mu = d[hi] - eh * eh / (dd + (dd >= 0 ? 1.0 : -1.0) * std::hypot(dd, eh));
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            // R = [[c, s], [-s, c]] on (k, k+1) with s x + c z = 0 zeroes the bulge (k-1, k+1);
            // for k = lo it brings in the shift
            const double r = std::hypot(x, z);
            const double c = r == 0.0 ? 1.0 : x / r, s = r == 0.0 ? 0.0 : -z / r;
            if (k > lo) e[k - 1] = r;
            const double p0 = d[k], p1 = d[k + 1], ek = e[k];
            d[k] = c * c * p0 - 2.0 * c * s * ek + s * s * p1;
            d[k + 1] = s * s * p0 + 2.0 * c * s * ek + c * c * p1;
            e[k] = c * s * (p0 - p1) + (c * c - s * s) * ek;
            if (k + 1 < hi) {
                const double f = e[k + 1];
                z = -s * f;            // the new bulge (k, k+2)
                e[k + 1] = c * f;
                x = e[k];
            }
            rotate(k, c, s);
        }
    }
    std::vector<double> ev(N);
    for (int j = 0; j < N; ++j) ev[j] = std::exp(p.tau * d[j]);
    // P = V diag(ev) V^T, entry (i, j) a weighted dot product of columns i and j of V^T, taken
    // from the rows of V
    std::vector<double> vr((size_t)N * N);
    for (int r = 0; r < N; ++r)
        for (int i = 0; i < N; ++i) vr[(size_t)i * N + r] = vt[(size_t)r * N + i];
    P->assign((size_t)N * N, 0.0);
    for (int i = 0; i < N; ++i) {
        const double* ri = &vr[(size_t)i * N];
        for (int r = 0; r < N; ++r) w[r] = ri[r] * ev[r];
        for (int j = i; j < N; ++j) {
            const double* rj = &vr[(size_t)j * N];
            double acc = 0.0;
            for (int r = 0; r < N; ++r) acc += w[r] * rj[r];
            (*P)[(size_t)i * N + j] = (*P)[(size_t)j * N + i] = acc;
        }
    }
    return std::string();
}

std::string build_energy_tables(const AxisParams& p, int log2e, EnergyTables* out) {
    const int N = p.n;
    if (N < 1) return "N must be >= 1";
    const int M = embed_length(N);
    if (M > kMaxEnergyLength) {
        char msg[128];
        snprintf(msg, sizeof msg, "N = %d exceeds the energy kernel's limit %d", N, kMaxEnergyLength / 2);
        return msg;
    }
    const std::vector<ld> b = first_column_B(p);
    // x^T B x = x'^T K x' for x' = x zero-padded to M and K the length-M circulant with
    // K[d mod M] = b_{|d|} (|d| < N; M >= 2N - 1 keeps the two ends apart), and by Parseval
    // x'^T K x' = (1/M) sum_m G[m] |X[m]|^2 with G[m] = b_0 + 2 sum_{d>=1} b_d cos(2 pi m d / M)
    int log2m = 0;
    while ((1 << log2m) < M) ++log2m;
    std::vector<ld> cosm(M);
    for (int r = 0; r < M; ++r) cosm[r] = cosl(2.0L * kPi * (ld)r / (ld)M);
    std::vector<double> G(M);
    for (int m = 0; m < M; ++m) {
        ld acc = b[0];
        long long r = m % M;
        for (int d = 1; d < N; ++d) {
            acc += 2.0L * b[d] * cosm[(size_t)r];
            r += m;
            if (r >= M) r -= M;
        }
        G[m] = (double)(acc / (ld)M);
    }
    EnergyTables& t = *out;
    t = EnergyTables();
    t.n = N;
    t.length = M;
    t.tw_re.resize(M);
    t.tw_im.resize(M);
    for (int m = 0; m < M; ++m) {
        const ld ang = 2.0L * kPi * (ld)m / (ld)M;
        t.tw_re[m] = (double)cosl(ang);
        t.tw_im[m] = (double)-sinl(ang);
    }
    t.gpos.resize(M);
    for (int q = 0; q < M; ++q) t.gpos[q] = G[embed_frequency(q, log2m, log2e)];
    return std::string();
}

std::string build_axis_tables(const AxisParams& p, int method, AxisTables* out, int log2e, bool diag2,
                              bool increment) {
    const int N = p.n;
    char msg[256];
    if (N < 1) return "N must be >= 1";
    if (!(p.alpha > 1.0 && p.alpha <= 2.0)) {
        snprintf(msg, sizeof msg, "alpha = %g is outside (1, 2]", p.alpha);
        return msg;
    }
    if (!(p.eps >= 0.0) || !std::isfinite(p.eps)) return "eps must be finite and >= 0";
    if (!(p.tau > 0.0) || !std::isfinite(p.tau)) return "tau must be finite and > 0";
    if (!(p.h > 0.0) || !std::isfinite(p.h)) return "h must be finite and > 0";

    AxisTables& t = *out;
    t = AxisTables();
    t.n = N;
    t.method = method;
    t.increment = increment;
    if (method == SFAC_METHOD_DIAG) {
        if (N > kMaxDiagLength) {
            snprintf(msg, sizeof msg, "N = %d exceeds the diagonal method's limit %d", N, kMaxDiagLength);
            return msg;
        }
        if (!factor_radices(N, &t.radices)) {
            snprintf(msg, sizeof msg, "N = %d has a prime factor above %d (use the embedded method)",
                     N, kMaxPrimeRadix);
            return msg;
        }
        t.length = N;
    } else if (method == SFAC_METHOD_EMBED) {
        int m = embed_length(N);
        if (m > kMaxEmbedLength) {
            snprintf(msg, sizeof msg, "N = %d exceeds the embedded method's limit %d", N, kMaxEmbedLength / 2);
            return msg;
        }
        factor_radices(m, &t.radices);
        t.length = m;
    } else {
        return "unknown method";
    }

    const std::vector<ld> b = first_column_B(p);

    // eqs. (C), (S)
    std::vector<ld> c(N), s(N);
    c[0] = s[0] = 0.5L * b[0];
    for (int k = 1; k < N; ++k) {
        c[k] = 0.5L * (b[k] + b[N - k]);
        s[k] = 0.5L * (b[k] - b[N - k]);
    }

    // Remark 1: spectra (real parts; the imaginary parts vanish by symmetry)
    // Angle indices (2 j k mod 2N and k (2j + 1) mod 2N) advance by a fixed step per term, kept
    // reduced by one conditional subtraction instead of a division per term.
    const std::vector<ld> cosn = half_turn_cosines(N);  // cos(pi r / N)
    const int twoN = 2 * N;
    auto advance = [](int& r, int step, int mod) {
        r += step;
        if (r >= mod) r -= mod;
    };
    std::vector<ld> lam(N), mu(N);
    for (int j = 0; j < N; ++j) {
        ld sl = 0, sm = 0;
        const int st1 = (int)((2LL * j) % twoN), st2 = (int)((2LL * j + 1) % twoN);
        int r1 = 0, r2 = 0;  // 2 j k and k (2j + 1), mod 2N, at k
        for (int k = 0; k < N; ++k) {
            sl += c[k] * cosn[r1];
            sm += s[k] * cosn[r2];
            advance(r1, st1, twoN);
            advance(r2, st2, twoN);
        }
        lam[j] = sl;
        mu[j] = sm;
    }
    // eigenvalues of the factors, or of the factors minus the identity (expm1 keeps the small
    // ones to full relative precision: |tau lambda_j| is small for the low frequencies)
    const ld tau = p.tau;
    std::vector<ld> ec(N), es(N);
    for (int j = 0; j < N; ++j) {
        ec[j] = increment ? expm1l(0.5L * tau * lam[j]) : expl(0.5L * tau * lam[j]);
        es[j] = increment ? expm1l(tau * mu[j]) : expl(tau * mu[j]);
    }

    const int L = t.length;
    t.tw_re.resize(L);
    t.tw_im.resize(L);
    for (int m = 0; m < L; ++m) {
        ld ang = 2.0L * kPi * (ld)m / (ld)L;
        t.tw_re[m] = (double)cosl(ang);
        t.tw_im[m] = (double)-sinl(ang);
    }

    if (method == SFAC_METHOD_DIAG) {
        t.scale_c.resize(N);
        t.scale_s.resize(N);
        t.psi_re.resize(N);
        t.psi_im.resize(N);
        for (int j = 0; j < N; ++j) {
            t.scale_c[j] = (double)(ec[j] / (ld)N);
            t.scale_s[j] = (double)(es[j] / (ld)N);
        }
        for (int k = 0; k < N; ++k) {
            ld ang = kPi * (ld)k / (ld)N;
            t.psi_re[k] = (double)cosl(ang);
            t.psi_im[k] = (double)-sinl(ang);
        }
        int A = 0, B = 0;
        if (diag2 && diag2_pair(N, &A, &B)) {
            // prime-factor index maps of the two-step kernel: thread b, register a holds position
            // (B a + A b) mod N; thread k1, register k2 holds frequency
            // (B (B^-1 mod A) k1 + A (A^-1 mod B) k2) mod N
            t.d2a = A;
            t.d2b = B;
            int binv = 1, ainv = 1;
            while ((B * binv) % A != 1 % A) ++binv;
            while ((A * ainv) % B != 1 % B) ++ainv;
            t.psi2_re.resize(N);
            t.psi2_im.resize(N);
            t.gpos_c.resize(N);
            t.gpos_s.resize(N);
            for (int b = 0; b < B; ++b)
                for (int a = 0; a < A; ++a) {
                    const int n = (B * a + A * b) % N;
                    t.psi2_re[b * A + a] = t.psi_re[n];
                    t.psi2_im[b * A + a] = t.psi_im[n];
                }
            for (int k1 = 0; k1 < A; ++k1)
                for (int k2 = 0; k2 < B; ++k2) {
                    const int k = (int)(((long long)B * binv * k1 + (long long)A * ainv * k2) % N);
                    t.gpos_c[k1 * B + k2] = t.scale_c[k];
                    t.gpos_s[k1 * B + k2] = t.scale_s[k];
                }
        }
    } else {
        // first columns of e^{tau/2 C} (circulant, gamma) and e^{tau S} (skew-circulant, sigma):
        // gamma_k = (1/N) sum_j e^{tau/2 lambda_j} cos(2 pi j k / N),
        // sigma_k = (1/N) sum_j e^{tau mu_j} cos(pi k (2j + 1) / N); both matrices are symmetric
        // Toeplitz, so entry (p, q) is gamma_{|p-q|} resp. sigma_{|p-q|}. In the increment form
        // ec / es hold the eigenvalues minus one and these are the columns of the factors minus
        // the identity (again symmetric Toeplitz).
        std::vector<ld> gam(N), sig(N);
        for (int k = 0; k < N; ++k) {
            ld sg = 0, ss = 0;
            const int st = (int)((2LL * k) % twoN);
            int r1 = 0, r2 = k % twoN;  // 2 j k and k (2j + 1), mod 2N, at j
            for (int j = 0; j < N; ++j) {
                sg += ec[j] * cosn[r1];
                ss += es[j] * cosn[r2];
                advance(r1, st, twoN);
                advance(r2, st, twoN);
            }
            gam[k] = sg / (ld)N;
            sig[k] = ss / (ld)N;
        }
        // length-M circular kernels g[d mod M] = col[|d|], |d| < N; their spectra are real:
        // G[m] = col[0] + 2 sum_{d=1}^{N-1} col[d] cos(2 pi m d / M); the 1/M of the inverse
        // transform is folded in.
        std::vector<ld> cosm(L);
        for (int r = 0; r < L; ++r) cosm[r] = cosl(2.0L * kPi * (ld)r / (ld)L);
        t.scale_c.resize(L);
        t.scale_s.resize(L);
        for (int m = 0; m < L; ++m) {
            ld gc = gam[0], gs = sig[0];
            const int st = m % L;
            int r = st;  // m d mod M, at d
            for (int d = 1; d < N; ++d) {
                const ld cs = cosm[r];
                gc += 2.0L * gam[d] * cs;
                gs += 2.0L * sig[d] * cs;
                advance(r, st, L);
            }
            t.scale_c[m] = (double)(gc / (ld)L);
            t.scale_s[m] = (double)(gs / (ld)L);
        }
        int log2m = 0;
        while ((1 << log2m) < L) ++log2m;
        t.gpos_c.resize(L);
        t.gpos_s.resize(L);
        for (int p = 0; p < L; ++p) {
            const int k = embed_frequency(p, log2m, log2e);
            t.gpos_c[p] = t.scale_c[k];
            t.gpos_s[p] = t.scale_s[k];
        }
    }
    return std::string();
}

}  // namespace sfac
