// Axis-pass kernels of the two-level Strang step (eqs. (hatv), (finalstrang), Remark 1).
//
// One pass handles every line of the state along one axis: it loads a tile of lines, packs
// two real lines into one complex line (the per-axis operator is real, so the real and
// imaginary parts are transformed independently), applies e^{tau/2 C} e^{tau S} e^{tau/2 C}
// by transforms in LDS, and stores the lines back in place. The first pass of a step applies
// the nonlinear half-step J^Q_{tau/2} (eq. (nonlinear_operator)) on load, the last pass applies
// it on store and records max |u| and non-finite values.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "sfac_diag2.hpp"
#include "sfac_embed.hpp"
#include "sfac_fft.hpp"
#include "sfac_kernels.hpp"

namespace sfac {

namespace {

// J^Q_{tau/2} v = v / sqrt(v^2 + (1 - v^2) e^{-tau}), with 1 - v^2 formed as (1 - v)(1 + v).
// e^{-tau} is carried as hi + lo in the state's type (lo = 0 for FP64): in FP32 the rounding of
// e^{-tau} would otherwise bias every half-step the same way.
// 1/sqrt(x) for x > 0. FP64: the hardware estimate refined by two Newton steps
// y <- y (3/2 - x y^2 / 2), each of which roughly doubles the number of correct bits. FP32:
// a correctly rounded square root and division.
__device__ __forceinline__ double recip_sqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-h * y, y, 0.5);
        y = fma(y, e, y);
    }
    return y;
}
__device__ __forceinline__ float recip_sqrt(float x) { return 1.0f / __builtin_sqrtf(x); }

template <typename T>
__device__ __forceinline__ T nonlinear_half_step(T v, T decay, T decay_lo) {
    const T one = (T)1;
    const T q = (one - v) * (one + v);
    return v * recip_sqrt(v * v + (q * decay + q * decay_lo));
}

// FP32 fast form for the register-resident kernels: hardware reciprocal square root estimate
// (inputs below the normal range scaled by 2^24, the result by 2^12) and one Newton step, within
// about one ulp at a third of the instructions of a correctly rounded square root and division.
// The exact flow maps [-1, 1] into itself (the discrete maximum principle of the nonlinear
// step); the estimate's rounding may land one ulp outside, so the result is put back for
// |v| <= 1 only, and values pushed past 1 by the linear step still show.
__device__ __forceinline__ float recip_sqrt_fast(float x) {
    const bool tiny = x < 1.17549435e-38f;
    const float y0 = __builtin_amdgcn_rsqf(tiny ? x * 16777216.0f : x);
    const float y = tiny ? y0 * 4096.0f : y0;
    const float h = 0.5f * x;
    const float e = fmaf(-h * y, y, 0.5f);
    return fmaf(y, e, y);
}
template <typename T>
__device__ __forceinline__ T nonlinear_half_step_fast(T v, T decay, T decay_lo) {
    if constexpr (sizeof(T) == 4) {
        const float q = (1.0f - v) * (1.0f + v);
        const float r = v * recip_sqrt_fast(v * v + (q * decay + q * decay_lo));
        return fabsf(v) <= 1.0f ? fminf(fmaxf(r, -1.0f), 1.0f) : r;
    } else {
        return nonlinear_half_step(v, decay, decay_lo);
    }
}

// The two real lines of a pair at one position: adjacent in memory on strided axes
// (lstride == 1), where one 2-element access (element-aligned, as the hardware allows) replaces
// two; a missing second line (two == false) reads as zero and is never touched.
template <typename T>
struct alignas(sizeof(T)) RealPair {
    T a, b;
};
template <typename T>
__device__ __forceinline__ void load_pair(const T* p, long long lstride, bool two, T& x, T& y) {
    if (lstride == 1 && two) {
        RealPair<T> v;
        __builtin_memcpy(&v, p, sizeof(v));
        x = v.a;
        y = v.b;
    } else {
        x = p[0];
        y = two ? p[lstride] : (T)0;
    }
}
template <typename T>
__device__ __forceinline__ void store_pair(T* p, long long lstride, bool two, T x, T y) {
    if (lstride == 1 && two) {
        const RealPair<T> v = {x, y};
        __builtin_memcpy(p, &v, sizeof(v));
    } else {
        p[0] = x;
        if (two) p[lstride] = y;
    }
}

template <int DIR, typename T>
__device__ __forceinline__ void run_stage(int R, const cplx<T>* src, cplx<T>* dst, int L, int Ns,
                                          int lines, const cplx<T>* tw) {
    switch (R) {
        case 2: stockham_stage<2, DIR>(src, dst, L, Ns, lines, tw); break;
        case 3: stockham_stage<3, DIR>(src, dst, L, Ns, lines, tw); break;
        case 4: stockham_stage<4, DIR>(src, dst, L, Ns, lines, tw); break;
        case 5: stockham_stage<5, DIR>(src, dst, L, Ns, lines, tw); break;
        case 7: stockham_stage<7, DIR>(src, dst, L, Ns, lines, tw); break;
        case 8: stockham_stage<8, DIR>(src, dst, L, Ns, lines, tw); break;
        case 9: stockham_stage<9, DIR>(src, dst, L, Ns, lines, tw); break;
        case 11: stockham_stage<11, DIR>(src, dst, L, Ns, lines, tw); break;
        case 13: stockham_stage<13, DIR>(src, dst, L, Ns, lines, tw); break;
        case 16: stockham_stage<16, DIR>(src, dst, L, Ns, lines, tw); break;
        case 17: stockham_stage<17, DIR>(src, dst, L, Ns, lines, tw); break;
        case 19: stockham_stage<19, DIR>(src, dst, L, Ns, lines, tw); break;
        case 23: stockham_stage<23, DIR>(src, dst, L, Ns, lines, tw); break;
        case 29: stockham_stage<29, DIR>(src, dst, L, Ns, lines, tw); break;
        case 31: stockham_stage<31, DIR>(src, dst, L, Ns, lines, tw); break;
        default: break;  // the host only plans the radices above
    }
}

// Full transform of `lines` lines; returns the buffer holding the result.
template <int DIR, typename T>
__device__ cplx<T>* transform(const PassDesc<T>& d, cplx<T>* cur, cplx<T>* other, int lines) {
    int Ns = 1;
    for (int s = 0; s < d.nst; ++s) {
        const int R = d.radix[s];
        run_stage<DIR>(R, cur, other, d.L, Ns, lines, d.tw);
        __syncthreads();
        cplx<T>* t = cur;
        cur = other;
        other = t;
        Ns *= R;
    }
    return cur;
}

// Wave-level reduction of the store statistics, then one atomic per wave.
template <typename T>
__device__ __forceinline__ void publish_stats(double vmax, unsigned int bad, const PassDesc<T>& d) {
    unsigned long long* smax = d.stat_max;
    unsigned int* sflags = d.stat_flags;
    for (int off = 32; off > 0; off >>= 1) {
        vmax = fmax(vmax, __shfl_xor(vmax, off));
        bad |= __shfl_xor(bad, off);
    }
    if ((threadIdx.x & 63) == 0) {
        if (vmax > 1.0) bad |= SFAC_FLAG_ABOVE_ONE;
        if (bad) atomicOr(sflags, bad);
        // atomics on one address from every wave serialise; the running maximum rarely grows
        // after the first step, so compare with the (possibly stale, never larger) stored value
        // first and only then update
        const unsigned long long bits = (unsigned long long)__double_as_longlong(vmax);
        if (bits > __atomic_load_n(smax, __ATOMIC_RELAXED)) atomicMax(smax, bits);
        // the per-step record (the maximum norm after every step, Sec. 5, Example 4): each
        // wavefront stores into its own slot, reduced after the step (no shared address)
        if (d.trace_part) d.trace_part[(size_t)blockIdx.x * d.trace_wpb + (threadIdx.x >> 6)] = bits;
    }
}

// Statistics of one stored pair: the largest finite |u| and the non-finite flag (the second
// value counts only when the pair holds two real lines).
template <typename T>
__device__ __forceinline__ void track_stats(const cplx<T>& z, bool two, double& vmax, unsigned int& bad) {
    const double ax = fabs((double)z.x), ay = two ? fabs((double)z.y) : 0.0;
    if (!(ax <= 1.7976931348623157e308) || !(ay <= 1.7976931348623157e308))
        bad |= SFAC_FLAG_NONFINITE;
    else
        vmax = fmax(vmax, fmax(ax, ay));
}

// The step boundary inside a pass that covers its axis twice (eq. (finalstrang) applied twice,
// the last pass of one step and the first of the next on the same axis): the closing half-step
// J^Q_{tau/2} of the first step, its statistics, and the opening half-step of the next. The
// values are exactly those the two separate passes would store and load again; a pair that
// holds one real line keeps zero in its second slot, as a fresh load gives it.
//
// Every half-step's input and result pass through an empty asm statement (as_stored), here and
// where the passes load and store: the compiler may otherwise fuse a product on one side of a
// half-step into the sums on the other (the transform's last product into 1 - v, the half-step's
// final product into the transform's first sums) wherever the two meet in one kernel, which
// would skip a rounding that a store and a load between two launches make.
template <typename T>
__device__ __forceinline__ T as_stored(T x) {
    asm volatile("" : "+v"(x));
    return x;
}
template <typename T>
__device__ __forceinline__ T nl_isolated(T v, T decay, T decay_lo) {
    return as_stored(nonlinear_half_step_fast(as_stored(v), decay, decay_lo));
}
template <typename T>
__device__ __forceinline__ cplx<T> step_boundary(cplx<T> z, bool two, T decay, T decay_lo, double& vmax,
                                                 unsigned int& bad) {
    z.x = nl_isolated(z.x, decay, decay_lo);
    z.y = two ? nl_isolated(z.y, decay, decay_lo) : (T)0;
    track_stats(z, two, vmax, bad);
    z.x = nl_isolated(z.x, decay, decay_lo);
    z.y = nl_isolated(z.y, decay, decay_lo);
    return z;
}

// keep: a third LDS buffer of lpb lines, used in the increment form only (the factor's input).
template <typename T>
__device__ __forceinline__ void run_tile(const PassDesc<T>& d, int tile, cplx<T>* buf0, cplx<T>* buf1, cplx<T>* keep) {
    const int N = d.N, L = d.L, lpb = d.lpb;
    const bool contiguous = d.inner == 1;
    long long first;       // first real line (row) or column of the tile
    long long avail;       // real lines available from `first`
    T* base;               // address of element 0 of real line `first`
    long long lstride;     // distance between adjacent real lines
    long long kstride;     // distance between adjacent elements of a line
    if (contiguous) {
        first = (long long)tile * 2 * lpb;
        avail = d.outer - first;
        base = d.u + first * N;
        lstride = N;
        kstride = 1;
    } else {
        const long long o = tile / d.tiles_per_outer;
        first = (long long)(tile % d.tiles_per_outer) * 2 * lpb;
        avail = d.inner - first;
        base = d.u + o * (long long)N * d.inner + first;
        lstride = 1;
        kstride = d.inner;
    }
    const int nreal = (int)(avail < 2 * lpb ? avail : 2 * lpb);
    const int lines = (nreal + 1) >> 1;
    const bool nl_in = d.nl_in != 0;
    const T decay = d.decay, decay_lo = d.decay_lo;

    // load (with zero padding to the transform length and a zero partner for an odd line)
    const int total = lines * L;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        int b, k;
        if (contiguous) {
            b = idx / L;
            k = idx - b * L;
        } else {
            k = idx / lines;
            b = idx - k * lines;
        }
        cplx<T> z = {(T)0, (T)0};
        if (k < N) {
            const T* p = base + (long long)(2 * b) * lstride + (long long)k * kstride;
            z.x = p[0];
            if (2 * b + 1 < nreal) z.y = p[lstride];
            if (nl_in) {
                z.x = nonlinear_half_step(z.x, decay, decay_lo);
                z.y = nonlinear_half_step(z.y, decay, decay_lo);
            }
        }
        buf0[b * L + k] = z;
    }
    __syncthreads();

    cplx<T>* cur = buf0;
    cplx<T>* other = buf1;
    const bool diag = d.method == 1;
    for (int f = 0; f < 3; ++f) {
        const Spec<T>* scale = f == 1 ? d.scale_s : d.scale_c;
        const bool skew = f == 1;
        if constexpr (increment_form<T>()) {   // every thread keeps (and later adds) its own elements
            for (int idx = threadIdx.x; idx < total; idx += blockDim.x) keep[idx] = cur[idx];
        }
        if (diag && skew) {  // x <- psi . x
            for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
                const int k = idx % L;
                cur[idx] = cmul(cur[idx], d.psi[k]);
            }
            __syncthreads();
        }
        cur = transform<-1>(d, cur, other, lines);
        other = cur == buf0 ? buf1 : buf0;
        for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
            const int k = idx % L;
            const Spec<T> sc = scale[k];
            cur[idx].x = spec_mul(cur[idx].x, sc);
            cur[idx].y = spec_mul(cur[idx].y, sc);
        }
        __syncthreads();
        cur = transform<+1>(d, cur, other, lines);
        other = cur == buf0 ? buf1 : buf0;
        if (diag && skew) {  // x <- conj(psi) . x
            for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
                const int k = idx % L;
                cur[idx] = cmulc(cur[idx], d.psi[k]);
            }
            __syncthreads();
        } else if (!diag) {  // embedded: keep the first N entries of the circular result
            for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
                const int k = idx % L;
                if (k >= N) cur[idx] = {(T)0, (T)0};
            }
            __syncthreads();
        }
        if constexpr (increment_form<T>()) {   // padding positions hold zero in both
            for (int idx = threadIdx.x; idx < total; idx += blockDim.x) cur[idx] = cur[idx] + keep[idx];
            __syncthreads();
        }
    }

    // store
    const bool nl_out = d.nl_out != 0;
    double vmax = 0.0;
    unsigned int bad = 0;
    const int stotal = lines * N;
    for (int idx = threadIdx.x; idx < stotal; idx += blockDim.x) {
        int b, k;
        if (contiguous) {
            b = idx / N;
            k = idx - b * N;
        } else {
            k = idx / lines;
            b = idx - k * lines;
        }
        cplx<T> z = cur[b * L + k];
        if (nl_out) {
            z.x = nonlinear_half_step(z.x, decay, decay_lo);
            z.y = nonlinear_half_step(z.y, decay, decay_lo);
        }
        T* p = base + (long long)(2 * b) * lstride + (long long)k * kstride;
        p[0] = z.x;
        const bool two = 2 * b + 1 < nreal;
        if (two) p[lstride] = z.y;
        if (nl_out) {
            const double ax = fabs((double)z.x), ay = two ? fabs((double)z.y) : 0.0;
            if (!(ax <= 1.7976931348623157e308) || !(ay <= 1.7976931348623157e308))
                bad |= SFAC_FLAG_NONFINITE;
            else
                vmax = fmax(vmax, fmax(ax, ay));
        }
    }
    if (nl_out) publish_stats(vmax, bad, d);
}

// Lines of one tile: a tile is 2*lpb real lines (rows of the contiguous axis, or adjacent
// columns of a strided one) packed pairwise into lpb complex lines.
template <typename T>
struct TileGeom {
    T* base;             // element 0 of the tile's first real line
    long long lstride;   // distance between adjacent real lines
    long long kstride;   // distance between adjacent elements of a line
    int nreal;           // real lines in this tile (<= 2 lpb)
    __device__ TileGeom(const PassDesc<T>& d, int tile) {
        long long first, avail;
        if (d.inner == 1) {
            first = (long long)tile * 2 * d.lpb;
            avail = d.outer - first;
            base = d.u + first * d.N;
            lstride = d.N;
            kstride = 1;
        } else {
            const long long o = tile / d.tiles_per_outer;
            first = (long long)(tile % d.tiles_per_outer) * 2 * d.lpb;
            avail = d.inner - first;
            base = d.u + o * (long long)d.N * d.inner + first;
            lstride = 1;
            kstride = d.inner;
        }
        nreal = (int)(avail < 2 * d.lpb ? avail : 2 * d.lpb);
    }
};

// Tile I/O of the embedded method through LDS (option `stage`). Every element of the tile makes
// one trip between HBM and its pair's LDS line; the walk puts adjacent threads on adjacent
// memory: along the line on the contiguous axis, across adjacent line pairs at one position on
// strided axes (a strided pass of one pair per block reads 16-byte runs per position; lpb pairs
// make runs of lpb x 16 bytes). Positions n < N of line pair l sit at the swizzled position n of
// LDS line l; a thread walks at most E/2 positions since N <= M/2. Threads beyond lpb lines (a
// batched launch sized for a larger descriptor) take no part.
template <typename T, int LOG2M, int LE, bool LOAD>
__device__ __forceinline__ void embed_stage(const PassDesc<T>& d, const TileGeom<T>& tg, cplx<T>* lds) {
    using G = EmbedGeom<LOG2M, LE>;
    const int lpb = d.lpb, tau = threadIdx.x;
    if (tau >= lpb * G::T) return;
    const bool contiguous = tg.kstride == 1;
    const int l = contiguous ? tau >> G::LOG2T : tau % lpb;
    const int n0 = contiguous ? tau & (G::T - 1) : tau / lpb;
    const bool x_in = 2 * l < tg.nreal, y_in = 2 * l + 1 < tg.nreal;
    if (!x_in) return;
    T* g = tg.base + 2LL * l * tg.lstride;
    cplx<T>* sl = lds + l * G::M;
    const int N = d.N;
#pragma unroll
    for (int j = 0; j < (G::E > 1 ? G::E / 2 : 1); ++j) {
        const int n = n0 + j * G::T;
        if (n < N) {
            if constexpr (LOAD) {
                cplx<T> z;
                load_pair(g + (long long)n * tg.kstride, tg.lstride, y_in, z.x, z.y);
                if (d.nl_in) {
                    z.x = nonlinear_half_step_fast(z.x, d.decay, d.decay_lo);
                    z.y = nonlinear_half_step_fast(z.y, d.decay, d.decay_lo);
                }
                sl[embed_swz<T, LOG2M>(n)] = z;
            } else {
                const cplx<T> z = sl[embed_swz<T, LOG2M>(n)];
                store_pair(g + (long long)n * tg.kstride, tg.lstride, y_in, z.x, z.y);
            }
        }
    }
}

// Embedded method, register-resident transforms of length 2^LOG2M; STAGE: tile I/O through LDS.
// TWICE: the pass covers its axis twice with a step boundary between (nl_mid).
// Always inlined: called out of line (as the compiler chose for the two-pass kernels with 16
// elements per thread in three radix passes), the two-pass kernel differed from two launches in
// the last bits, and its LDS exchanges go through generic pointers.
template <typename T, int LOG2M, int LE, bool STAGE, bool TWICE = false>
__device__ __forceinline__ void run_embed_tile(const PassDesc<T>& d, int tile, cplx<T>* lds) {
    using G = EmbedGeom<LOG2M, LE>;
    using Line = EmbedLine<T, LOG2M, LE>;
    const int line = threadIdx.x >> G::LOG2T;
    const int t = threadIdx.x & (G::T - 1);
    const TileGeom<T> tg(d, tile);
    const int N = d.N;
    const bool act = 2 * line < tg.nreal;
    const bool two = 2 * line + 1 < tg.nreal;
    const T decay = d.decay, decay_lo = d.decay_lo;
    Line L;
    L.load_twiddles(d.tw, t);
    cplx<T>* ln = lds + line * G::M;
    if constexpr (STAGE) {
        embed_stage<T, LOG2M, LE, true>(d, tg, lds);
        __syncthreads();
    }
    T* const own = tg.base + (long long)(2 * line) * tg.lstride;   // this thread's line pair
    constexpr int R0 = G::R(0);
#pragma unroll
    for (int i = 0; i < G::E / R0; ++i)
#pragma unroll
        for (int k = 0; k < R0; ++k) {
            const int n = Line::nat(t, i, k);
            cplx<T> z = {(T)0, (T)0};
            if ((R0 < 2 || k < R0 / 2) && act && n < N) {
                if constexpr (STAGE) {
                    z = ln[embed_swz<T, LOG2M>(n)];
                } else {
                    load_pair(own + (long long)n * tg.kstride, tg.lstride, two, z.x, z.y);
                    if (d.nl_in) {
                        z.x = nl_isolated(z.x, decay, decay_lo);
                        z.y = nl_isolated(z.y, decay, decay_lo);
                    }
                }
            }
            L.a[i * R0 + k] = z;
        }
    double vmax = 0.0;
    unsigned int bad = 0;
    // Unrolled: the second pass must see the same compile-time zeros (the padding registers) as
    // a pass that loads its tile, so that the compiler simplifies and fuses its arithmetic the
    // same way and the values stay bitwise those of two launches.
    // FP64 also seals the three factors: every register enters and leaves them through as_stored,
    // so that the block is compiled from the same opaque inputs in a single and a two-pass kernel.
    constexpr int reps = TWICE ? 2 : 1;
    constexpr bool SEAL = sizeof(T) == 8;
#pragma unroll
    for (int r = 0; r < reps; ++r) {
        if (r == 1) {
#pragma unroll
            for (int i = 0; i < G::E / R0; ++i)
#pragma unroll
                for (int k = 0; k < R0; ++k)
                    if ((R0 < 2 || k < R0 / 2) && act && Line::nat(t, i, k) < N)
                        L.a[i * R0 + k] = step_boundary(L.a[i * R0 + k], two, decay, decay_lo, vmax, bad);
        }
        if constexpr (SEAL) {
#pragma unroll
            for (int e = 0; e < G::E; ++e) {
                L.a[e].x = as_stored(L.a[e].x);
                L.a[e].y = as_stored(L.a[e].y);
            }
        }
        L.factor(d.gpos_c, ln, t, N);
        L.factor(d.gpos_s, ln, t, N);
        L.factor(d.gpos_c, ln, t, N);
        if constexpr (SEAL) {
#pragma unroll
            for (int e = 0; e < G::E; ++e) {
                L.a[e].x = as_stored(L.a[e].x);
                L.a[e].y = as_stored(L.a[e].y);
            }
        }
    }
    if constexpr (STAGE) __syncthreads();   // the last exchange's reads are done before the staging writes
#pragma unroll
    for (int i = 0; i < G::E / R0; ++i)
#pragma unroll
        for (int k = 0; k < R0; ++k) {
            const int n = Line::nat(t, i, k);
            if ((R0 < 2 || k < R0 / 2) && act && n < N) {
                cplx<T> z = L.a[i * R0 + k];
                if (d.nl_out) {
                    z.x = nl_isolated(z.x, decay, decay_lo);
                    z.y = nl_isolated(z.y, decay, decay_lo);
                    track_stats(z, two, vmax, bad);
                }
                if constexpr (STAGE)
                    ln[embed_swz<T, LOG2M>(n)] = z;
                else
                    store_pair(own + (long long)n * tg.kstride, tg.lstride, two, z.x, z.y);
            }
        }
    if constexpr (STAGE) {
        __syncthreads();
        embed_stage<T, LOG2M, LE, false>(d, tg, lds);
    }
    if (d.nl_out || TWICE) publish_stats(vmax, bad, d);
}

template <typename T, int A, int B, bool LOAD>
__device__ __forceinline__ void stage_tile(const TileGeom<T>& tg, int lpb, cplx<T>* lds) {
    constexpr int P = A > B ? A : B, N = A * B, J = N / P;
    constexpr int LS = diag2_line_stride(A, B, sizeof(cplx<T>));
    const int tau = threadIdx.x;
    if (tau >= lpb * P) return;
    const bool contiguous = tg.kstride == 1;
    const int l = contiguous ? tau / P : tau % lpb;
    const int n0 = contiguous ? tau - l * P : tau / lpb;
    const bool x_in = 2 * l < tg.nreal, y_in = 2 * l + 1 < tg.nreal;
    const T* gx = tg.base + 2 * l * tg.lstride + n0 * tg.kstride;
    const long long step = (long long)P * tg.kstride;
    cplx<T>* sl = lds + l * LS + n0;
    if constexpr (LOAD) {
        cplx<T> v[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (x_in) {
                load_pair(gx + j * step, tg.lstride, y_in, v[j].x, v[j].y);
            } else {
                v[j].x = (T)0;
                v[j].y = (T)0;
            }
        }
#pragma unroll
        for (int j = 0; j < J; ++j) sl[j * P] = v[j];
    } else {
        cplx<T> v[J];
#pragma unroll
        for (int j = 0; j < J; ++j) v[j] = sl[j * P];
        T* gw = const_cast<T*>(gx);
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (x_in) store_pair(gw + j * step, tg.lstride, y_in, v[j].x, v[j].y);
    }
}

// Diagonal method, register-resident two-step transforms of length N = A B. The tile goes
// through LDS on the way in and out (the prime-factor layout scatters a thread's positions).
// TWICE: the pass covers its axis twice with a step boundary between (nl_mid).
template <typename T, int A, int B, bool WA, bool TWICE = false>
__device__ __forceinline__ void run_diag2_tile(const PassDesc<T>& d, int tile, cplx<T>* lds) {
    using G = Diag2Geom<A, B>;
    using Line = Diag2Line<T, A, B, WA>;
    int line, t;
    if constexpr (WA) {
        // lines never straddle wavefronts; lanes beyond LPW P idle (t = P takes no part)
        const int lane = threadIdx.x & 63, lw = lane / G::P;
        line = (threadIdx.x >> 6) * G::LPW + (lw < G::LPW ? lw : G::LPW - 1);
        t = lw < G::LPW ? lane - lw * G::P : G::P;
    } else {
        line = threadIdx.x / G::P;
        t = threadIdx.x - line * G::P;
    }
    const TileGeom<T> tg(d, tile);
    const bool act = 2 * line < tg.nreal && t < G::P;
    const bool two = 2 * line + 1 < tg.nreal;
    const T decay = d.decay, decay_lo = d.decay_lo;
    stage_tile<T, A, B, true>(tg, d.lpb, lds);
    __syncthreads();
    Line L;
    cplx<T>* ln = lds + line * diag2_line_stride(A, B, sizeof(cplx<T>));
    if (t < B) {
#pragma unroll
        for (int k = 0; k < A; ++k) {
            cplx<T> z = {(T)0, (T)0};
            if (act) {
                z = ln[G::pos(t, k)];
                if (d.nl_in) {
                    z.x = nl_isolated(z.x, decay, decay_lo);
                    z.y = nl_isolated(z.y, decay, decay_lo);
                }
            }
            L.a[k] = z;
        }
    }
    double vmax = 0.0;
    unsigned int bad = 0;
    constexpr int reps = TWICE ? 2 : 1;
#pragma unroll 1
    for (int r = 0; r < reps; ++r) {
        if (r == 1 && t < B && act) {
#pragma unroll
            for (int k = 0; k < A; ++k) L.a[k] = step_boundary(L.a[k], two, decay, decay_lo, vmax, bad);
        }
        L.factors(d.gpos_c, d.gpos_s, d.psi2, ln, t);
    }
    __syncthreads();   // the last exchange's reads are done before the staging writes
    if (t < B && act) {
#pragma unroll
        for (int k = 0; k < A; ++k) {
            cplx<T> z = L.a[k];
            if (d.nl_out) {
                z.x = nl_isolated(z.x, decay, decay_lo);
                z.y = nl_isolated(z.y, decay, decay_lo);
                track_stats(z, two, vmax, bad);
            }
            ln[G::pos(t, k)] = z;
        }
    }
    __syncthreads();
    stage_tile<T, A, B, false>(tg, d.lpb, lds);
    if (d.nl_out || TWICE) publish_stats(vmax, bad, d);
}

// blockIdx -> tile, grouping neighbouring tiles on one XCD (blocks are dealt round-robin to
// the 8 XCDs, so block b runs on XCD b % 8): tiles that share cache lines then share an L2.
__device__ __forceinline__ int xcd_tile(int block, int ntiles) {
    const int per = (ntiles + 7) >> 3;
    return (block & 7) * per + (block >> 3);
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads) axis_pass_single(PassDesc<T> d) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* buf0 = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* buf1 = buf0 + d.lpb * d.L;
    const int tile = d.xcd_remap ? xcd_tile(blockIdx.x, d.ntiles) : (int)blockIdx.x;
    if (tile >= d.ntiles) return;
    run_tile(d, tile, buf0, buf1, buf1 + d.lpb * d.L);
}

// Block size bound of an embedded-method kernel: 256 threads, or one line when a line has more
// threads (512 at four elements each); staged kernels: at least two lines (embed_stage_block).
// Above 256 threads the second bound asks for two wavefronts per SIMD (a 1024-thread bound
// alone keeps the kernel within 128 registers, four wavefronts per SIMD).
constexpr int embed_max_block(int log2m, int le, bool stage) {
    const int t = 1 << (log2m - embed_log2e(log2m, le));
    return stage ? embed_stage_block(t) : (t > kBlockThreads ? t : kBlockThreads);
}
// FP32 blocks above 256 threads with at most 8 elements per thread ask for four wavefronts per
// SIMD (at most 128 VGPRs), so that two 512-thread blocks share a CU: a batched launch of many
// lines then keeps twice the wavefronts in flight.
template <typename T>
constexpr int embed_min_waves(int log2m, int le, bool stage) {
    return embed_max_block(log2m, le, stage) > kBlockThreads ? (sizeof(T) == 4 && le <= 3 ? 4 : 2) : 1;
}
#define SFAC_EMBED_BOUNDS(LOG2M, LE, STAGE)                   \
    __launch_bounds__(embed_max_block(LOG2M, LE, STAGE), (embed_min_waves<T>(LOG2M, LE, STAGE)))

// TWICE: two passes over the axis in one launch (descriptors with nl_mid), a distinct kernel so
// that the single passes keep their register allocation.
template <typename T, int LOG2M, int LE, bool STAGE, bool TWICE>
__global__ void SFAC_EMBED_BOUNDS(LOG2M, LE, STAGE) embed_pass_single(PassDesc<T> d) {
    extern __shared__ unsigned char smem_raw[];
    const int tile = d.xcd_remap ? xcd_tile(blockIdx.x, d.ntiles) : (int)blockIdx.x;
    if (tile >= d.ntiles) return;
    run_embed_tile<T, LOG2M, LE, STAGE, TWICE>(d, tile, reinterpret_cast<cplx<T>*>(smem_raw));
}

// The instance of a grouped launch that owns block b (the last entry whose first block is at
// most b) and its descriptor, with the state pointer of the launch; *local gets the block's
// index within that instance's pass.
template <typename T>
__device__ __forceinline__ PassDesc<T> group_desc(const GroupArgs<T>& g, int b, int* local) {
    int lo = 0, hi = g.n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (g.start[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    PassDesc<T> d = *g.desc[lo];
    d.u = g.u[lo];
    *local = b - g.start[lo];
    return d;
}

// Several instances with the same transform length in one launch (batched form).
template <typename T, int LOG2M, int LE, bool STAGE, bool TWICE>
__global__ void SFAC_EMBED_BOUNDS(LOG2M, LE, STAGE) embed_pass_multi(const GroupArgs<T> g) {
    extern __shared__ unsigned char smem_raw[];
    int local;
    const PassDesc<T> d = group_desc(g, blockIdx.x, &local);
    const int tile = d.xcd_remap ? xcd_tile(local, d.ntiles) : local;
    if (tile >= d.ntiles) return;
    // the block has the group's largest size; threads beyond d.lpb lines hold no line (their
    // LDS rows lie inside the block's allocation) and only take part in the barriers
    run_embed_tile<T, LOG2M, LE, STAGE, TWICE>(d, tile, reinterpret_cast<cplx<T>*>(smem_raw));
}

// Waves per SIMD the register budget is cut for: three (at most 168 VGPRs). Every pair fits
// without spilling (FP64 15 x 17: 156 VGPRs); with six lines per block or the wavefront-aligned
// layout the FP64 15 x 17 tiles also fit three wavefronts per SIMD in the LDS.
template <typename T, int A, int B, bool WA>
constexpr int diag2_min_waves() {
    return 3;
}

template <typename T, int A, int B, bool WA, bool TWICE>
__global__ void __launch_bounds__(kBlockThreads, (diag2_min_waves<T, A, B, WA>())) diag2_pass_single(PassDesc<T> d) {
    extern __shared__ unsigned char smem_raw[];
    const int tile = d.xcd_remap ? xcd_tile(blockIdx.x, d.ntiles) : (int)blockIdx.x;
    if (tile >= d.ntiles) return;
    run_diag2_tile<T, A, B, WA, TWICE>(d, tile, reinterpret_cast<cplx<T>*>(smem_raw));
}

template <typename T, int A, int B, bool WA, bool TWICE>
__global__ void __launch_bounds__(kBlockThreads, (diag2_min_waves<T, A, B, WA>())) diag2_pass_multi(const GroupArgs<T> g) {
    extern __shared__ unsigned char smem_raw[];
    int local;
    const PassDesc<T> d = group_desc(g, blockIdx.x, &local);
    const int tile = d.xcd_remap ? xcd_tile(local, d.ntiles) : local;
    if (tile >= d.ntiles) return;
    run_diag2_tile<T, A, B, WA, TWICE>(d, tile, reinterpret_cast<cplx<T>*>(smem_raw));
}

template <typename T, int A, int B, bool WA>
const void* diag2_fn_w(bool multi, bool twice) {
    if (multi)
        return twice ? reinterpret_cast<const void*>(&diag2_pass_multi<T, A, B, WA, true>)
                     : reinterpret_cast<const void*>(&diag2_pass_multi<T, A, B, WA, false>);
    return twice ? reinterpret_cast<const void*>(&diag2_pass_single<T, A, B, WA, true>)
                 : reinterpret_cast<const void*>(&diag2_pass_single<T, A, B, WA, false>);
}
template <typename T, int A, int B>
const void* diag2_fn_ab(bool multi, bool wave, bool twice) {
    return wave ? diag2_fn_w<T, A, B, true>(multi, twice) : diag2_fn_w<T, A, B, false>(multi, twice);
}

// the (A, B) pairs the host may plan (see diag2_pair); wave: the wavefront-aligned layout
template <typename T>
const void* diag2_fn(int a, int b, bool multi, bool wave, bool twice) {
    switch (a * 64 + b) {
        case 3 * 64 + 5: return diag2_fn_ab<T, 3, 5>(multi, wave, twice);
        case 5 * 64 + 7: return diag2_fn_ab<T, 5, 7>(multi, wave, twice);
        case 7 * 64 + 9: return diag2_fn_ab<T, 7, 9>(multi, wave, twice);
        case 9 * 64 + 11: return diag2_fn_ab<T, 9, 11>(multi, wave, twice);
        case 11 * 64 + 13: return diag2_fn_ab<T, 11, 13>(multi, wave, twice);
        case 13 * 64 + 15: return diag2_fn_ab<T, 13, 15>(multi, wave, twice);
        case 15 * 64 + 17: return diag2_fn_ab<T, 15, 17>(multi, wave, twice);
        case 5 * 64 + 9: return diag2_fn_ab<T, 5, 9>(multi, wave, twice);
        case 7 * 64 + 11: return diag2_fn_ab<T, 7, 11>(multi, wave, twice);
        default: return nullptr;
    }
}

// kernel of one (transform length, elements per thread, staging); LE = 2 (M = 64 to 2048), 3 or 4
template <typename T, int LOG2M, int LE, bool STAGE>
const void* embed_fn_k(bool multi, bool twice) {
    if (multi)
        return twice ? reinterpret_cast<const void*>(&embed_pass_multi<T, LOG2M, LE, STAGE, true>)
                     : reinterpret_cast<const void*>(&embed_pass_multi<T, LOG2M, LE, STAGE, false>);
    return twice ? reinterpret_cast<const void*>(&embed_pass_single<T, LOG2M, LE, STAGE, true>)
                 : reinterpret_cast<const void*>(&embed_pass_single<T, LOG2M, LE, STAGE, false>);
}
template <typename T, int LOG2M, bool STAGE>
const void* embed_fn_le(int le, bool multi, bool twice) {
    if (le == 2) {
        if constexpr (LOG2M >= 6 && LOG2M <= 11) return embed_fn_k<T, LOG2M, 2, STAGE>(multi, twice);
        return nullptr;
    }
    if (le == 3) return embed_fn_k<T, LOG2M, 3, STAGE>(multi, twice);
    return embed_fn_k<T, LOG2M, 4, STAGE>(multi, twice);
}
// staged kernels exist for M >= 64 (lines of at least 32 points)
template <typename T, int LOG2M>
const void* embed_fn_lm(int le, bool multi, bool stage, bool twice) {
    if (!stage) return embed_fn_le<T, LOG2M, false>(le, multi, twice);
    if constexpr (LOG2M >= 6) return embed_fn_le<T, LOG2M, true>(le, multi, twice);
    return nullptr;
}

template <typename T>
const void* embed_fn(int log2m, int le, bool multi, bool stage, bool twice) {
    switch (log2m) {
        case 1: return embed_fn_lm<T, 1>(le, multi, stage, twice);
        case 2: return embed_fn_lm<T, 2>(le, multi, stage, twice);
        case 3: return embed_fn_lm<T, 3>(le, multi, stage, twice);
        case 4: return embed_fn_lm<T, 4>(le, multi, stage, twice);
        case 5: return embed_fn_lm<T, 5>(le, multi, stage, twice);
        case 6: return embed_fn_lm<T, 6>(le, multi, stage, twice);
        case 7: return embed_fn_lm<T, 7>(le, multi, stage, twice);
        case 8: return embed_fn_lm<T, 8>(le, multi, stage, twice);
        case 9: return embed_fn_lm<T, 9>(le, multi, stage, twice);
        case 10: return embed_fn_lm<T, 10>(le, multi, stage, twice);
        case 11: return embed_fn_lm<T, 11>(le, multi, stage, twice);
        case 12: return embed_fn_lm<T, 12>(le, multi, stage, twice);
        default: return nullptr;
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads) axis_pass_multi(const GroupArgs<T> g) {
    extern __shared__ unsigned char smem_raw[];
    int local;
    const PassDesc<T> d = group_desc(g, blockIdx.x, &local);
    const int tile = d.xcd_remap ? xcd_tile(local, d.ntiles) : local;
    if (tile >= d.ntiles) return;
    cplx<T>* buf0 = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* buf1 = buf0 + d.lpb * d.L;
    run_tile(d, tile, buf0, buf1, buf1 + d.lpb * d.L);
}

// Discrete energy (Sec. 5, Example 5), one axis. A thread block holds lpb line pairs packed as
// x + i y. Their zero-padded length-M transform X gives sum_m G[m] |X[m]|^2 = x^T B x + y^T B y:
// the cross terms of the packing cancel between m and M - m because G is symmetric. The loads
// also sum the double-well term when d.nl_in is set (once per element: on one axis only).
// Sums are kept in FP64 whatever T, reduced over each wavefront and added with one atomic each.
template <typename T, int LOG2M>
__global__ void __launch_bounds__(kBlockThreads) energy_pass(PassDesc<T> d) {
    constexpr int LE = energy_log2e(LOG2M);
    using G = EmbedGeom<LOG2M, LE>;
    using Line = EmbedLine<T, LOG2M, LE>;
    extern __shared__ unsigned char smem_raw[];
    const int tile = d.xcd_remap ? xcd_tile(blockIdx.x, d.ntiles) : (int)blockIdx.x;
    if (tile >= d.ntiles) return;
    const int line = threadIdx.x >> G::LOG2T;
    const int t = threadIdx.x & (G::T - 1);
    const TileGeom<T> tg(d, tile);
    const int N = d.N;
    const bool act = 2 * line < tg.nreal;
    const bool two = 2 * line + 1 < tg.nreal;
    Line L;
    L.load_twiddles(d.tw, t);
    const T* own = tg.base + (long long)(2 * line) * tg.lstride;
    constexpr int R0 = G::R(0);
    double well = 0.0;
#pragma unroll
    for (int i = 0; i < G::E / R0; ++i)
#pragma unroll
        for (int k = 0; k < R0; ++k) {
            const int n = Line::nat(t, i, k);
            cplx<T> z = {(T)0, (T)0};
            if ((R0 < 2 || k < R0 / 2) && act && n < N) {
                load_pair(own + (long long)n * tg.kstride, tg.lstride, two, z.x, z.y);
                if (d.nl_in) {
                    const double qx = (double)z.x * (double)z.x - 1.0;
                    const double qy = (double)z.y * (double)z.y - 1.0;
                    well += 0.25 * qx * qx + (two ? 0.25 * qy * qy : 0.0);
                }
            }
            L.a[i * R0 + k] = z;
        }
    cplx<T>* ln = reinterpret_cast<cplx<T>*>(smem_raw) + line * G::M;
    L.template fwd_from<0>(ln, t);
    constexpr int S = G::NST - 1;
    constexpr int R = G::R(S);
    double quad = 0.0;
#pragma unroll
    for (int i = 0; i < G::E / R; ++i)
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const Spec<T> g = d.gpos_c[embed_pos<LOG2M, LE, S>(t, i, k)];
            double gv;
            if constexpr (sizeof(T) == 8)
                gv = (double)g.v;
            else
                gv = (double)g.hi + (double)g.lo;
            const cplx<T> z = L.a[i * R + k];
            quad += gv * ((double)z.x * (double)z.x + (double)z.y * (double)z.y);
        }
    for (int off = 32; off > 0; off >>= 1) {
        quad += __shfl_xor(quad, off);
        well += __shfl_xor(well, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&d.energy[0], quad);
        if (d.nl_in) atomicAdd(&d.energy[1], well);
    }
}

template <typename T>
const void* energy_fn(int log2m) {
    switch (log2m) {
        case 1: return reinterpret_cast<const void*>(&energy_pass<T, 1>);
        case 2: return reinterpret_cast<const void*>(&energy_pass<T, 2>);
        case 3: return reinterpret_cast<const void*>(&energy_pass<T, 3>);
        case 4: return reinterpret_cast<const void*>(&energy_pass<T, 4>);
        case 5: return reinterpret_cast<const void*>(&energy_pass<T, 5>);
        case 6: return reinterpret_cast<const void*>(&energy_pass<T, 6>);
        case 7: return reinterpret_cast<const void*>(&energy_pass<T, 7>);
        case 8: return reinterpret_cast<const void*>(&energy_pass<T, 8>);
        case 9: return reinterpret_cast<const void*>(&energy_pass<T, 9>);
        case 10: return reinterpret_cast<const void*>(&energy_pass<T, 10>);
        case 11: return reinterpret_cast<const void*>(&energy_pass<T, 11>);
        case 12: return reinterpret_cast<const void*>(&energy_pass<T, 12>);
        default: return nullptr;
    }
}

}  // namespace

template <typename T>
int pass_blocks(const PassDesc<T>& d) {
    return d.xcd_remap ? 8 * ((d.ntiles + 7) / 8) : d.ntiles;
}

template <typename T>
hipError_t launch_axis_pass(const PassDesc<T>& d, size_t lds_bytes, hipStream_t stream) {
    const int blocks = pass_blocks(d);
    if (blocks <= 0) return hipSuccess;
    if (d.method == 2 || (d.method == 1 && d.d2a > 0)) {
        const bool twice = d.nl_mid != 0;
        const void* fn = d.method == 2 ? embed_fn<T>(d.log2m, d.log2e, false, d.stage != 0, twice)
                                       : diag2_fn<T>(d.d2a, d.d2b, false, d.d2wave != 0, twice);
        if (!fn) return hipErrorInvalidValue;
        void* args[] = {const_cast<PassDesc<T>*>(&d)};
        return hipLaunchKernel(fn, dim3(blocks), dim3(d.threads), args, lds_bytes, stream);
    }
    hipLaunchKernelGGL(axis_pass_single<T>, dim3(blocks), dim3(kBlockThreads), lds_bytes, stream, d);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_axis_pass_multi(int kind, int variant, int threads, const GroupArgs<T>& args, size_t lds_bytes,
                                  hipStream_t stream) {
    if (args.n < 1 || args.n > kGroupSlots) return hipErrorInvalidValue;
    const int total_blocks = args.start[args.n];
    if (total_blocks <= 0) return hipSuccess;
    if (kind == 1 || kind == 2) {
        const bool twice = variant >= kTwiceVariant;
        const int v = variant % kTwiceVariant;
        const void* fn = kind == 1 ? embed_fn<T>((v % 128) / 8, v % 8, true, v >= 128, twice)
                                   : diag2_fn<T>((v % 4096) / 64, v % 64, true, v >= 4096, twice);
        if (!fn) return hipErrorInvalidValue;
        void* kargs[] = {const_cast<GroupArgs<T>*>(&args)};
        return hipLaunchKernel(fn, dim3(total_blocks), dim3(threads), kargs, lds_bytes, stream);
    }
    hipLaunchKernelGGL(axis_pass_multi<T>, dim3(total_blocks), dim3(kBlockThreads), lds_bytes, stream, args);
    return hipGetLastError();
}

namespace {
// Dense FP64 product C = X Y (row-major, per batch index), on the matrix cores: v_mfma_f64_16x16x4 takes
// A (16 x 4) as lane l -> row l % 16, k = l / 16, B (4 x 16) as lane l -> column l % 16,
// k = l / 16, and returns D (16 x 16) in four registers, register i of lane l holding row
// 4 i + l / 16, column l % 16. A block of four wavefronts owns a 32 x 32 tile of C, one 16 x 16
// quarter per wavefront; K advances in slabs of 32 staged through LDS (X transposed, so both
// operands are read along m or n by consecutive lanes), the next slab loaded into registers
// while the current one is multiplied. Every load and store is guarded, so any M, N, K work.
//
// Tiles to XCDs: workgroup L of a launch runs on XCD L mod 8, and each XCD has its own L2. The
// tile grid of one batch index is cut into gy x gx rectangles of rm x rn tiles, one per XCD,
// with (gy, gx) chosen so that an XCD reads as few row bands of X and column bands of Y as
// possible (an operand shared by every batch index costs nothing: it stays in the L2 across the
// batch); inside a rectangle the shorter side runs fastest, so workgroups dispatched one after
// another share the band of the longer side while they read it. Slots beyond the grid exit.
// A batch of at least 8 products sharing X (rm == 0) is dealt by whole products instead:
// product b on XCD b mod 8, its tiles one after another, so each Y slab is read by one L2.
constexpr int kGemmThreads = 256, kXcds = 8;
typedef double double4_t __attribute__((ext_vector_type(4)));

// W x W matrix-core tiles of 16 x 16 per wavefront: the block tile is 32 W x 32 W, K advances in
// slabs of BK.
template <int W, int BK>
__global__ void __launch_bounds__(kGemmThreads) exact_gemm(const double* __restrict__ X, const double* __restrict__ Y,
                                                           double* __restrict__ C, int M, int N, int K, long long ldx,
                                                           long long ldy, long long ldc, long long sx, long long sy,
                                                           long long sc, int tiles_m, int tiles_n, int gx, int rm,
                                                           int rn, int batch) {
    constexpr int kTile = 32 * W;
    __shared__ double xs[2][BK][kTile + 1];   // xs[k][m]
    __shared__ double ys[2][BK][kTile + 1];   // ys[k][n]
    const int xcd = (int)(blockIdx.x % kXcds), slot = (int)(blockIdx.x / kXcds);
    int tm, tn;
    long long b;
    if (rm == 0) {   // whole products per XCD
        const int per = tiles_m * tiles_n;
        b = (long long)(slot / per) * kXcds + xcd;
        tm = (slot % per) % tiles_m;
        tn = (slot % per) / tiles_m;
        if (b >= batch) return;   // the whole block, before any barrier
    } else {
        const bool n_fast = rn <= rm;
        tm = (xcd / gx) * rm + (n_fast ? slot / rn : slot % rm);
        tn = (xcd % gx) * rn + (n_fast ? slot % rn : slot / rm);
        b = blockIdx.y;
        if (tm >= tiles_m || tn >= tiles_n) return;   // the whole block, before any barrier
    }
    X += b * sx;
    Y += b * sy;
    C += b * sc;
    const int m0 = tm * kTile, n0 = tn * kTile;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = (wave >> 1) * 16 * W, wn = (wave & 1) * 16 * W;
    constexpr int kPer = kTile * BK / kGemmThreads;   // elements of each slab per thread
    double xr[kPer], yr[kPer];
    auto load = [&](int k0) {
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int idx = t + r * kGemmThreads;
            const int mm = idx / BK, kk = idx % BK;          // consecutive threads along a row of X
            const int gm = m0 + mm, gk = k0 + kk;
            xr[r] = (gm < M && gk < K) ? X[(long long)gm * ldx + gk] : 0.0;
            const int kk2 = idx / kTile, nn = idx % kTile;   // along a row of Y
            const int gk2 = k0 + kk2, gn = n0 + nn;
            yr[r] = (gk2 < K && gn < N) ? Y[(long long)gk2 * ldy + gn] : 0.0;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int idx = t + r * kGemmThreads;
            xs[buf][idx % BK][idx / BK] = xr[r];
            ys[buf][idx / kTile][idx % kTile] = yr[r];
        }
    };
    double4_t acc[W][W];
#pragma unroll
    for (int i = 0; i < W; ++i)
#pragma unroll
        for (int j = 0; j < W; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
    load(0);
    stash(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < K; k0 += BK) {
        const bool more = k0 + BK < K;
        if (more) load(k0 + BK);
#pragma unroll
        for (int k4 = 0; k4 < BK; k4 += 4) {
            double a[W], bb[W];
#pragma unroll
            for (int i = 0; i < W; ++i) a[i] = xs[buf][k4 + (lane >> 4)][wm + 16 * i + (lane & 15)];
#pragma unroll
            for (int j = 0; j < W; ++j) bb[j] = ys[buf][k4 + (lane >> 4)][wn + 16 * j + (lane & 15)];
#pragma unroll
            for (int i = 0; i < W; ++i)
#pragma unroll
                for (int j = 0; j < W; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
        }
        if (more) stash(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const int gn = n0 + wn + 16 * j + (lane & 15);
#pragma unroll
        for (int i = 0; i < W; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + 16 * i + 4 * r + (lane >> 4);
                if (gm < M && gn < N) C[(long long)gm * ldc + gn] = acc[i][j][r];
            }
    }
}

// With `halves` = 2 the launch is a step boundary: the closing half-step (whose values the
// statistics see), then the next step's opening half-step on the value as stored.
__global__ void __launch_bounds__(kExactNlThreads) exact_nl(double* dst, const double* src, long long n, double decay,
                                                            int stats, int halves, PassDesc<double> d) {
    const long long i = (long long)blockIdx.x * kExactNlThreads + threadIdx.x;
    double vmax = 0.0;
    unsigned int bad = 0;
    if (i < n) {
        double z = nonlinear_half_step(src[i], decay, 0.0);
        const double az = fabs(z);
        if (!(az <= 1.7976931348623157e308))
            bad |= SFAC_FLAG_NONFINITE;
        else
            vmax = az;
        if (halves == 2) z = nonlinear_half_step(as_stored(z), decay, 0.0);
        dst[i] = z;
    }
    if (stats) publish_stats(vmax, bad, d);
}
}  // namespace

hipError_t launch_exact_gemm(const double* X, const double* Y, double* C, int M, int N, int K, long long ldx,
                             long long ldy, long long ldc, long long sx, long long sy, long long sc, int batch,
                             hipStream_t stream) {
    if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
    // 64 x 64 block tiles (2 x 2 matrix-core tiles per wavefront, half the LDS reads per product)
    // where they still give every SIMD several wavefronts (at least 8 blocks per CU); 32 x 32
    // otherwise (on 1023^2 the 64 x 64 tiles leave one wavefront per SIMD, and 32 x 64 tiles
    // two, and both are slower)
    const long long big = (long long)((M + 63) / 64) * ((N + 63) / 64) * batch;
    const int tile = big >= 8LL * 256 ? 64 : 32;
    const int tiles_m = (M + tile - 1) / tile, tiles_n = (N + tile - 1) / tile;
    const bool x_shared = sx == 0 && batch > 1, y_shared = sy == 0 && batch > 1;
    int gx = 1, rm = 0, rn = 0, best = 0;
    for (int g = 1; g <= kXcds; g *= 2) {   // gx column groups, kXcds / gx row groups
        const int m = (tiles_m + kXcds / g - 1) / (kXcds / g), n = (tiles_n + g - 1) / g;
        const int cost = (x_shared ? 0 : m) + (y_shared ? 0 : n);
        if (rm == 0 || cost < best || (cost == best && m + n < rm + rn)) {
            gx = g;
            rm = m;
            rn = n;
            best = cost;
        }
    }
    // grid.x a multiple of 8: workgroup (x, b) runs on XCD x mod 8 for every batch index b
    dim3 grid((unsigned)kXcds * rm * rn, batch, 1);
    if (x_shared && batch >= kXcds) {   // whole products per XCD (rm = 0 selects it)
        grid = dim3((unsigned)kXcds * tiles_m * tiles_n * ((batch + kXcds - 1) / kXcds), 1, 1);
        rm = rn = 0;
    }
    if (tile == 64)
        hipLaunchKernelGGL((exact_gemm<2, 16>), grid, dim3(kGemmThreads), 0, stream, X, Y, C, M, N, K, ldx, ldy, ldc,
                           sx, sy, sc, tiles_m, tiles_n, gx, rm, rn, batch);
    else
        hipLaunchKernelGGL((exact_gemm<1, 32>), grid, dim3(kGemmThreads), 0, stream, X, Y, C, M, N, K, ldx, ldy, ldc,
                           sx, sy, sc, tiles_m, tiles_n, gx, rm, rn, batch);
    return hipGetLastError();
}

hipError_t launch_exact_nl(double* dst, const double* src, long long n, double decay, bool stats, int halves,
                           const PassDesc<double>& d, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    if (halves != 1 && halves != 2) return hipErrorInvalidValue;
    const long long blocks = (n + kExactNlThreads - 1) / kExactNlThreads;
    hipLaunchKernelGGL(exact_nl, dim3((unsigned)blocks), dim3(kExactNlThreads), 0, stream, dst, src, n, decay,
                       stats ? 1 : 0, halves, d);
    return hipGetLastError();
}

namespace {
constexpr int kCollectThreads = 1024;
__global__ void __launch_bounds__(kCollectThreads) trace_collect(unsigned long long* parts, long long nparts,
                                                                 unsigned long long* rec, long long* step,
                                                                 long long cap) {
    __shared__ unsigned long long wave_max[kCollectThreads / 64];
    unsigned long long m = 0;
    for (long long i = threadIdx.x; i < nparts; i += kCollectThreads) {
        m = m > parts[i] ? m : parts[i];
        parts[i] = 0;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off);
        m = m > o ? m : o;
    }
    if ((threadIdx.x & 63) == 0) wave_max[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kCollectThreads / 64; ++w) m = m > wave_max[w] ? m : wave_max[w];
        const long long k = *step;
        if (k < cap) rec[k] = m;
        atomicAdd(reinterpret_cast<unsigned long long*>(step), 1ull);
    }
}
}  // namespace

hipError_t launch_trace_collect(unsigned long long* parts, long long nparts, unsigned long long* rec, long long* step,
                                long long cap, hipStream_t stream) {
    hipLaunchKernelGGL(trace_collect, dim3(1), dim3(kCollectThreads), 0, stream, parts, nparts, rec, step, cap);
    return hipGetLastError();
}

namespace {
// An empty one-wavefront kernel whose name carries a number: launched around the timed launches
// of sfac_plan_time_passes (the axis, 1..3) and sfac_plan_time_fused (kFusedMark + the axis),
// it tells a kernel trace or counter record which launches the dispatches that follow are
// (0: the timed launches are over).
template <int AXIS>
__global__ void __launch_bounds__(64) pass_timing_mark() {}
}  // namespace

namespace {
__global__ void __launch_bounds__(64) zero_words(unsigned int* p, int words) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < words) p[i] = 0u;
}
}  // namespace

hipError_t launch_zero_words(unsigned int* p, int words, hipStream_t stream) {
    if (words <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_words, dim3((words + 63) / 64), dim3(64), 0, stream, p, words);
    return hipGetLastError();
}

hipError_t launch_timing_mark(int axis, hipStream_t stream) {
    switch (axis) {
        case 0: hipLaunchKernelGGL(pass_timing_mark<0>, dim3(1), dim3(64), 0, stream); break;
        case 1: hipLaunchKernelGGL(pass_timing_mark<1>, dim3(1), dim3(64), 0, stream); break;
        case 2: hipLaunchKernelGGL(pass_timing_mark<2>, dim3(1), dim3(64), 0, stream); break;
        case 3: hipLaunchKernelGGL(pass_timing_mark<3>, dim3(1), dim3(64), 0, stream); break;
        case kFusedMark + 1: hipLaunchKernelGGL(pass_timing_mark<kFusedMark + 1>, dim3(1), dim3(64), 0, stream); break;
        case kFusedMark + 2: hipLaunchKernelGGL(pass_timing_mark<kFusedMark + 2>, dim3(1), dim3(64), 0, stream); break;
        case kFusedMark + 3: hipLaunchKernelGGL(pass_timing_mark<kFusedMark + 3>, dim3(1), dim3(64), 0, stream); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_energy_pass(const PassDesc<T>& d, size_t lds_bytes, hipStream_t stream) {
    const int blocks = pass_blocks(d);
    if (blocks <= 0) return hipSuccess;
    const void* fn = energy_fn<T>(d.log2m);
    if (!fn) return hipErrorInvalidValue;
    void* args[] = {const_cast<PassDesc<T>*>(&d)};
    return hipLaunchKernel(fn, dim3(blocks), dim3(d.threads), args, lds_bytes, stream);
}

// The limit is a per-kernel attribute of the process: it only ever rises, so that a plan made
// later with a smaller need cannot take LDS away from the launches of an earlier one.
template <typename T>
hipError_t allow_lds(size_t lds_bytes) {
    static std::mutex lock;
    static size_t granted = 64 * 1024;
    std::lock_guard<std::mutex> guard(lock);
    if (lds_bytes <= granted) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&axis_pass_single<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    for (int lg = 1; lg <= 12; ++lg)
        for (int le = 2; le <= 4; ++le)
            for (int multi = 0; multi < 2; ++multi)
                for (int stage = 0; stage < 2; ++stage)
                    for (int twice = 0; twice < 2; ++twice) {
                        const void* fn = embed_fn<T>(lg, le, multi, stage, twice);
                        if (!fn) continue;
                        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
                        if (e != hipSuccess) return e;
                    }
    for (int lg = 1; lg <= 12; ++lg) {
        e = hipFuncSetAttribute(energy_fn<T>(lg), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    for (int a = 3; a <= 17; ++a)
        for (int b = a; b <= 17; ++b)
            for (int multi = 0; multi < 2; ++multi)
                for (int wave = 0; wave < 2; ++wave)
                    for (int twice = 0; twice < 2; ++twice) {
                        const void* fn = diag2_fn<T>(a, b, multi, wave, twice);
                        if (!fn) continue;
                        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
                        if (e != hipSuccess) return e;
                    }
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&axis_pass_multi<T>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e == hipSuccess) granted = lds_bytes;
    return e;
}

template int pass_blocks<double>(const PassDesc<double>&);
template int pass_blocks<float>(const PassDesc<float>&);
template hipError_t launch_axis_pass<double>(const PassDesc<double>&, size_t, hipStream_t);
template hipError_t launch_axis_pass<float>(const PassDesc<float>&, size_t, hipStream_t);
template hipError_t launch_axis_pass_multi<double>(int, int, int, const GroupArgs<double>&, size_t, hipStream_t);
template hipError_t launch_axis_pass_multi<float>(int, int, int, const GroupArgs<float>&, size_t, hipStream_t);
template hipError_t launch_energy_pass<double>(const PassDesc<double>&, size_t, hipStream_t);
template hipError_t launch_energy_pass<float>(const PassDesc<float>&, size_t, hipStream_t);
template hipError_t allow_lds<double>(size_t);
template hipError_t allow_lds<float>(size_t);

}  // namespace sfac
