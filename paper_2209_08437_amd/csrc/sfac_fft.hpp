// Device-side building blocks: complex arithmetic, compile-time trigonometric constants,
// small DFT kernels (radices 2..16 by power-of-two recursion, odd composite lengths with coprime
// factors by the prime-factor algorithm, other odd lengths up to 31 by the symmetric direct
// form) and a Stockham stage over lines held in local data share (LDS).
//
// Transform convention: forward (DIR = -1) is y_j = sum_k x_k e^{-2 pi i j k / L}; inverse
// (DIR = +1) uses e^{+2 pi i j k / L} without the 1/L, which the caller folds into its tables.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

namespace sfac {

// Aligned to its size so that LDS and global accesses of one element are single 16-byte
// (double) or 8-byte (float) operations.
template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T x, y;
};

// An eigenvalue-factor (spectrum) table entry. FP64 holds the value. FP32 holds the value
// rounded to float and the float remainder, and multiplies as a hi + lo pair (one more FMA), so
// the table adds no rounding of its own: the same rounded factor applied every step would
// otherwise give an error that grows linearly with the number of steps.
template <typename T>
struct Spec {
    T v;
};
template <>
struct Spec<float> {
    float hi, lo;
};
__host__ __device__ inline Spec<double> make_spec_double(double v) { return {v}; }
__host__ __device__ inline Spec<float> make_spec_float(double v) {
    const float hi = (float)v;
    return {hi, (float)(v - (double)hi)};
}
template <typename T>
__host__ __device__ inline Spec<T> make_spec(double v);
template <>
__host__ __device__ inline Spec<double> make_spec<double>(double v) { return make_spec_double(v); }
template <>
__host__ __device__ inline Spec<float> make_spec<float>(double v) { return make_spec_float(v); }

// FP32 passes apply every factor K in increment form, x + (K - I) x, from tables of K - I: the
// transforms then round the increment, which is small against x wherever the state is smooth
// (the low frequencies that carry it have eigenvalue factors near one), instead of x itself.
// FP64 passes apply K directly: their rounding is far below the method's error already, and the
// kept input would cost the FP64 register kernels a wavefront per SIMD.
template <typename T>
constexpr bool increment_form() { return sizeof(T) == sizeof(float); }

// a * g
__device__ __forceinline__ double spec_mul(double a, Spec<double> g) { return a * g.v; }
__device__ __forceinline__ float spec_mul(float a, Spec<float> g) { return __builtin_fmaf(a, g.lo, a * g.hi); }

template <typename T>
__device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) {
    return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) {
    return {a.x - b.x, a.y - b.y};
}
// a * b
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// multiply by DIR * i
template <int DIR, typename T>
__device__ __forceinline__ cplx<T> mul_i(cplx<T> a) {
    if constexpr (DIR < 0)
        return {a.y, -a.x};
    else
        return {-a.y, a.x};
}

// Orders the LDS accesses of one wavefront: its lanes execute in lockstep and its LDS operations
// complete in issue order, so only the compiler must be kept from moving them across.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------- compile-time trigonometry
// cos and sin of 2 pi p / q with exact rational reduction to the first octant, then a Taylor
// series at |x| <= pi/4 (terms to x^29; truncation far below one unit in the last place).
namespace ct {
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double sin_series(double x) {
    double x2 = x * x, term = x, sum = x;
    for (int n = 1; n < 15; ++n) {
        term *= -x2 / (double)((2 * n) * (2 * n + 1));
        sum += term;
    }
    return sum;
}
constexpr double cos_series(double x) {
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int n = 1; n < 15; ++n) {
        term *= -x2 / (double)((2 * n - 1) * (2 * n));
        sum += term;
    }
    return sum;
}
constexpr double sin_turn(long long p, long long q);
constexpr double cos_turn(long long p, long long q) {
    p %= q;
    if (p < 0) p += q;
    if (2 * p > q) p = q - p;                              // cos(2 pi (1 - f)) = cos(2 pi f)
    if (4 * p > q) return -cos_turn(q - 2 * p, 2 * q);     // f in (1/4, 1/2]
    if (8 * p > q) return sin_turn(q - 4 * p, 4 * q);      // f in (1/8, 1/4]
    return cos_series(2.0 * kPi * (double)p / (double)q);
}
constexpr double sin_turn(long long p, long long q) {
    p %= q;
    if (p < 0) p += q;
    if (2 * p > q) return -sin_turn(q - p, q);             // sin(2 pi (1 - f)) = -sin(2 pi f)
    if (4 * p > q) return sin_turn(q - 2 * p, 2 * q);      // sin(2 pi (1/2 - f)) = sin(2 pi f)
    if (8 * p > q) return cos_turn(q - 4 * p, 4 * q);      // sin(2 pi f) = cos(2 pi (1/4 - f))
    return sin_series(2.0 * kPi * (double)p / (double)q);
}
}  // namespace ct

// a * e^{DIR 2 pi i K / R}
template <int K, int R, int DIR, typename T>
__device__ __forceinline__ cplx<T> twiddle(cplx<T> a) {
    constexpr int k = K % R;
    if constexpr (k == 0) {
        return a;
    } else if constexpr (4 * k == R) {
        return mul_i<DIR>(a);
    } else if constexpr (2 * k == R) {
        return {-a.x, -a.y};
    } else if constexpr (4 * k == 3 * R) {
        return mul_i<-DIR>(a);
    } else {
        constexpr double c = ct::cos_turn(k, R);
        constexpr double s = DIR * ct::sin_turn(k, R);
        return {a.x * (T)c - a.y * (T)s, a.x * (T)s + a.y * (T)c};
    }
}

// ------------------------------------------------------------------ power-of-two DFTs
template <int R, int DIR, typename T>
struct DftPow2;

template <int DIR, typename T>
struct DftPow2<1, DIR, T> {
    static __device__ __forceinline__ void run(cplx<T>*) {}
};

template <int R, int DIR, typename T, int... K>
__device__ __forceinline__ void pow2_combine(cplx<T>* a, const cplx<T>* e, const cplx<T>* o,
                                             std::integer_sequence<int, K...>) {
    (
        [&] {
            const cplx<T> t = twiddle<K, R, DIR>(o[K]);
            a[K] = e[K] + t;
            a[K + R / 2] = e[K] - t;
        }(),
        ...);
}

template <int R, int DIR, typename T>
struct DftPow2 {
    static __device__ __forceinline__ void run(cplx<T>* a) {
        cplx<T> e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            e[i] = a[2 * i];
            o[i] = a[2 * i + 1];
        }
        DftPow2<R / 2, DIR, T>::run(e);
        DftPow2<R / 2, DIR, T>::run(o);
        pow2_combine<R, DIR>(a, e, o, std::make_integer_sequence<int, R / 2>{});
    }
};

// Radix-R DFT whose inputs R/2 .. R-1 are zero: even outputs are the half-length DFT of the
// nonzero inputs, odd outputs the half-length DFT of those inputs times e^{DIR 2 pi i n / R}.
template <int R, int DIR, typename T, int... K>
__device__ __forceinline__ void half_in_twiddle(cplx<T>* o, const cplx<T>* a, std::integer_sequence<int, K...>) {
    ((o[K] = twiddle<K, R, DIR>(a[K])), ...);
}
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_half_input(cplx<T>* a) {
    if constexpr (R == 1) {
        return;
    } else {
        cplx<T> e[R / 2], o[R / 2];
#pragma unroll
        for (int n = 0; n < R / 2; ++n) e[n] = a[n];
        half_in_twiddle<R, DIR>(o, a, std::make_integer_sequence<int, R / 2>{});
        DftPow2<R / 2, DIR, T>::run(e);
        DftPow2<R / 2, DIR, T>::run(o);
#pragma unroll
        for (int m = 0; m < R / 2; ++m) {
            a[2 * m] = e[m];
            a[2 * m + 1] = o[m];
        }
    }
}

// Radix-R DFT of which only outputs 0 .. R/2-1 are needed (the others are left undefined):
// y_n = DFT_{R/2}(even inputs)_n + e^{DIR 2 pi i n / R} DFT_{R/2}(odd inputs)_n.
template <int R, int DIR, typename T, int... K>
__device__ __forceinline__ void half_out_combine(cplx<T>* a, const cplx<T>* e, const cplx<T>* o,
                                                 std::integer_sequence<int, K...>) {
    ((a[K] = e[K] + twiddle<K, R, DIR>(o[K])), ...);
}
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_half_output(cplx<T>* a) {
    if constexpr (R == 1) {
        return;
    } else {
        cplx<T> e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            e[i] = a[2 * i];
            o[i] = a[2 * i + 1];
        }
        DftPow2<R / 2, DIR, T>::run(e);
        DftPow2<R / 2, DIR, T>::run(o);
        half_out_combine<R, DIR>(a, e, o, std::make_integer_sequence<int, R / 2>{});
    }
}

// ------------------------------------------------------------------------ odd DFTs
// y_j = a_0 + sum_k p_k cos(2 pi j k / R) + DIR i sum_k m_k sin(2 pi j k / R), k = 1..H,
// with p_k = a_k + a_{R-k}, m_k = a_k - a_{R-k}; y_{R-j} flips the sign of the sine part.
template <int R, int J, int K, typename T>
__device__ __forceinline__ void odd_acc(cplx<T>& A, cplx<T>& B, const cplx<T>* p, const cplx<T>* m) {
    if constexpr (K <= (R - 1) / 2) {
        constexpr double c = ct::cos_turn((long long)J * K % R, R);
        constexpr double s = ct::sin_turn((long long)J * K % R, R);
        A.x += p[K - 1].x * (T)c;
        A.y += p[K - 1].y * (T)c;
        B.x += m[K - 1].x * (T)s;
        B.y += m[K - 1].y * (T)s;
        odd_acc<R, J, K + 1>(A, B, p, m);
    }
}

template <int R, int DIR, int J, typename T>
__device__ __forceinline__ void odd_out(cplx<T>* y, cplx<T> a0, const cplx<T>* p, const cplx<T>* m) {
    if constexpr (J <= (R - 1) / 2) {
        cplx<T> A = a0, B = {(T)0, (T)0};
        odd_acc<R, J, 1>(A, B, p, m);
        const cplx<T> iB = mul_i<DIR>(B);
        y[J] = A + iB;
        y[R - J] = A - iB;
        odd_out<R, DIR, J + 1>(y, a0, p, m);
    }
}

// In place: every input is folded into p, m (and a0) before the first output is written.
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_odd(cplx<T>* a) {
    constexpr int H = (R - 1) / 2;
    cplx<T> p[H], m[H];
    const cplx<T> a0 = a[0];
    cplx<T> y0 = a0;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        p[k - 1] = a[k] + a[R - k];
        m[k - 1] = a[k] - a[R - k];
        y0 = y0 + p[k - 1];
    }
    odd_out<R, DIR, 1>(a, a0, p, m);
    a[0] = y0;
}

// Odd R = R1 R2 with coprime R1, R2 > 1: R1 is the full power of R's smallest prime factor
// (0 when R has no such split: a prime or a prime power).
constexpr int pfa_split(int r) {
    if (r % 2 == 0) return 0;
    for (int p = 3; p * p <= r; p += 2)
        if (r % p == 0) {
            int q = 1;
            while (r % p == 0) {
                r /= p;
                q *= p;
            }
            return r > 1 ? q : 0;
        }
    return 0;
}
constexpr int mod_inverse(int a, int m) {
    for (int x = 1; x < m; ++x)
        if ((a * x) % m == 1) return x;
    return 1;
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cplx<T>* a);

// Prime-factor (Good-Thomas) DFT of length R1 R2, gcd(R1, R2) = 1: input index
// n = (R2 n1 + R1 n2) mod R, output index k = (R2 (R2^-1 mod R1) k1 + R1 (R1^-1 mod R2) k2) mod R
// turn the length-R DFT into R2 DFTs of length R1 and R1 of length R2 with no twiddles.
template <int R1, int R2, int DIR, typename T>
__device__ __forceinline__ void dft_pfa(cplx<T>* a) {
    constexpr int R = R1 * R2;
    constexpr int i2 = mod_inverse(R2 % R1, R1), i1 = mod_inverse(R1 % R2, R2);
    cplx<T> u[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) u[n2][n1] = a[(R2 * n1 + R1 * n2) % R];
        dft<R1, DIR>(u[n2]);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        cplx<T> v[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) v[n2] = u[n2][k1];
        dft<R2, DIR>(v);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) a[(R2 * i2 * k1 + R1 * i1 * k2) % R] = v[k2];
    }
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cplx<T>* a) {
    if constexpr ((R & (R - 1)) == 0)
        DftPow2<R, DIR, T>::run(a);
    else if constexpr (pfa_split(R) > 0)
        dft_pfa<pfa_split(R), R / pfa_split(R), DIR>(a);
    else
        dft_odd<R, DIR>(a);
}

// ---------------------------------------------------------------- Stockham stage in LDS
// One radix-R pass of a self-sorting (Stockham) transform over `lines` lines of length L
// stored line after line (stride L) in src; results go to dst. Ns is the product of the radices
// of the earlier passes. tw[m] = e^{-2 pi i m / L}.
template <int R, int DIR, typename T>
__device__ __forceinline__ void stockham_stage(const cplx<T>* __restrict__ src, cplx<T>* __restrict__ dst,
                                               int L, int Ns, int lines,
                                               const cplx<T>* __restrict__ tw) {
    const int nb = L / R;
    const int twstep = L / (Ns * R);
    const int total = lines * nb;
    for (int w = threadIdx.x; w < total; w += blockDim.x) {
        const int b = w / nb;
        const int j = w - b * nb;
        const int k = j % Ns;
        const cplx<T>* s = src + b * L;
        cplx<T> a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = s[j + r * nb];
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const cplx<T> wv = tw[r * k * twstep];
                a[r] = DIR < 0 ? cmul(a[r], wv) : cmulc(a[r], wv);
            }
        }
        dft<R, DIR>(a);
        cplx<T>* dd = dst + b * L + (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dd[r * Ns] = a[r];
    }
}

}  // namespace sfac
