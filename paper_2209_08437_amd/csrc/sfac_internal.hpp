// Internal declarations shared by the host table builder, the kernels and the runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sfac.h"

namespace sfac {

constexpr int kMaxStages = 12;
constexpr int kMaxDiagLength = 4096;   // largest N for the length-N (diagonal) method
constexpr int kMaxEmbedLength = 4096;  // largest M for the embedded method (N <= 2048)
constexpr int kMaxPrimeRadix = 31;     // largest prime factor the mixed-radix transform handles

// One axis of one instance, as the host builds it (FP64 values).
struct AxisTables {
    int n = 0;                  // interior nodes N on this axis
    int method = 0;             // SFAC_METHOD_DIAG or SFAC_METHOD_EMBED
    int length = 0;             // transform length: N (diag) or M (embed)
    std::vector<int> radices;   // stage radices, product == length
    // twiddles e^{-2 pi i m / length}, m < length
    std::vector<double> tw_re, tw_im;
    // diag: e^{tau/2 lambda_j}/N and e^{tau mu_j}/N (length N)
    // embed: spectra of the Toeplitz kernels of e^{tau/2 C} and e^{tau S}, divided by M (length M)
    std::vector<double> scale_c, scale_s;
    // diag only: psi_k = e^{-i pi k / N}
    std::vector<double> psi_re, psi_im;
    // embed only: scale_c / scale_s permuted to the digit-reversed positions of the
    // register-resident transform (position p holds frequency embed_frequency(p));
    // two-step diagonal kernel (N = A B, prime-factor maps):
    // gpos[k1 B + k2] = scale[(B (B^-1 mod A) k1 + A (A^-1 mod B) k2) mod N]
    std::vector<double> gpos_c, gpos_s;
    // two-step diagonal kernel only: A, B and psi2[b A + a] = psi_{(B a + A b) mod N}
    int d2a = 0, d2b = 0;
    std::vector<double> psi2_re, psi2_im;
    // increment form: scale_c / scale_s (and their permutations) describe e^{tau/2 C} - I and
    // e^{tau S} - I (expm1 of the eigenvalue exponents); the kernels add the factor's input back
    bool increment = false;
};

// Factor pairs N = A * B handled by the register-resident diagonal kernel (false if none).
bool diag2_pair(int n, int* a, int* b);

// Frequency index held at in-place position p after all decimation-in-frequency passes of the
// register-resident power-of-two transform of length 2^log2m with at most 2^log2e elements per
// thread.
int embed_frequency(int p, int log2m, int log2e);

// Per-axis parameters of the method.
struct AxisParams {
    int n;
    double alpha, eps, tau, h;
};

// Builds the tables for one axis. Returns an empty string on success, else an error message.
// `method` is SFAC_METHOD_DIAG or SFAC_METHOD_EMBED (AUTO is resolved by the caller); for the
// embedded method `log2e` (3 or 4) selects the radix-pass schedule the position tables follow.
// `increment` builds the tables of the factors minus the identity (AxisTables::increment).
std::string build_axis_tables(const AxisParams& p, int method, AxisTables* out, int log2e = 4,
                              bool diag2 = true, bool increment = false);

// Factorisation of n into the supported radices (largest first); empty if n has a prime
// factor above kMaxPrimeRadix. n == 1 yields an empty list and returns true.
bool factor_radices(int n, std::vector<int>* radices);

// Default method for (n, dtype): the choice the library makes for SFAC_METHOD_AUTO.
int auto_method(int n, sfac_dtype dt);

// Smallest power of two >= 2n - 1 (at least 2).
int embed_length(int n);

// Tables of the energy kernel (discrete energy of Example 5, Sec. 5) for one axis: the
// length-M transform twiddles and the spectrum of B's circulant embedding divided by M, stored
// in the transform's last-pass position order (embed_frequency with the kernel's log2e).
constexpr int kMaxEnergyLength = 4096;
struct EnergyTables {
    int n = 0;
    int length = 0;
    std::vector<double> tw_re, tw_im;
    std::vector<double> gpos;
};
std::string build_energy_tables(const AxisParams& p, int log2e, EnergyTables* out);

// e^{tau B} for one axis (eq. (linear_operator) per axis: the exact exponential of the one-level
// scheme, eq. (strang)), a dense symmetric N x N matrix in row-major order, from the symmetric
// eigendecomposition of B (Householder tridiagonal reduction, implicit shifted QR). Returns an
// error message if the QR iteration does not converge.
constexpr int kMaxExactLength = 1024;
std::string build_exact_exponential(const AxisParams& p, std::vector<double>* P);

}  // namespace sfac
