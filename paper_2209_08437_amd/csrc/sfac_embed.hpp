// Register-resident axis pass for the embedded method (power-of-two transform length M).
//
// Each complex line (two real lines packed as real and imaginary parts) is held by T = M/E
// threads, E = min(2^LE, M) elements per thread (LE = 2, 3 or 4: more threads per line and more
// radix passes, or fewer threads and more registers; the plan picks per length and problem size). A length-M transform is an in-place
// decimation-in-frequency Cooley-Tukey pass sequence with radices R_0..R_{NST-1} (<= 16); the
// inverse runs the conjugate-transposed passes in reverse order (decimation in time), so the
// forward output (digit-reversed positions) is consumed where it lies and the inverse output
// comes back in natural order in exactly the registers the next forward transform reads: the
// only data movement between passes is one LDS exchange between consecutive radix passes.
// Per factor: forward transform, multiply by the kernel spectrum (stored on the host in the
// same digit-reversed position order), inverse transform, keep the first N entries.
// The pass twiddles of every thread are the same for all six transforms of a pass, so they
// are loaded once into registers.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "sfac_fft.hpp"

namespace sfac {

// Radix passes of a length-2^log2m transform with at most 2^log2e elements per thread: as few
// passes as possible, bits spread evenly, larger radices first.
constexpr int embed_log2e(int log2m, int log2e_max) { return log2m < log2e_max ? log2m : log2e_max; }
constexpr int embed_stages(int log2m, int log2e_max) {
    return log2m <= log2e_max ? 1 : (log2m + log2e_max - 1) / log2e_max;
}
constexpr int embed_bits(int log2m, int log2e_max, int s) {
    return log2m / embed_stages(log2m, log2e_max) + (s < log2m % embed_stages(log2m, log2e_max) ? 1 : 0);
}

template <int LOG2M, int LOG2E_MAX = 4>
struct EmbedGeom {
    static constexpr int M = 1 << LOG2M;
    static constexpr int LOG2E = embed_log2e(LOG2M, LOG2E_MAX);
    static constexpr int E = 1 << LOG2E;
    static constexpr int LOG2T = LOG2M - LOG2E;
    static constexpr int T = 1 << LOG2T;
    static constexpr int NST = embed_stages(LOG2M, LOG2E_MAX);
    static constexpr int bits(int s) { return embed_bits(LOG2M, LOG2E_MAX, s); }
    static constexpr int R(int s) { return 1 << bits(s); }
    // log2 of the stride S_s between the elements of one radix-R_s butterfly
    static constexpr int log2S(int s) {
        int acc = LOG2M;
        for (int q = 0; q <= s; ++q) acc -= bits(q);
        return acc;
    }
    // log2 of M / B_s, B_s = S_s R_s the span of a stage-s block (= product of earlier radices)
    static constexpr int log2Pre(int s) {
        int acc = 0;
        for (int q = 0; q < s; ++q) acc += bits(q);
        return acc;
    }
    // log2 of the butterflies each thread holds at pass s
    static constexpr int log2I(int s) { return LOG2E - bits(s); }
    // log2 of the wavefronts (64 threads) one line spans; 0 when a line fits in one wavefront
    static constexpr int LOG2W = LOG2T > 6 ? LOG2T - 6 : 0;
    // first pass whose butterflies leave the top LOG2W position bits alone (those bits are
    // butterfly bits of earlier passes only)
    static constexpr int SLOC = [] {
        int s = 1;
        while (s < NST && log2Pre(s) < LOG2W) ++s;
        return s;
    }();
    // the exchange between passes a and b stays inside one wavefront
    static constexpr bool local(int a, int b) { return LOG2W == 0 || (a >= SLOC && b >= SLOC); }
    // threads of one line (the block holds whole lines)
    static constexpr int max_block = T > 256 ? T : 256;
};

// Butterfly index of slot i of thread t at pass S. Before pass SLOC it is t + i T. From pass
// SLOC on the wavefront bits of t move to the top, above the slot bits, so that the top position
// bits name the wavefront; they are butterfly bits of passes before SLOC only, so the exchanges
// between passes >= SLOC stay inside one wavefront and need no workgroup barrier.
template <int LOG2M, int LE, int S>
__device__ __forceinline__ int embed_butterfly(int t, int i) {
    using G = EmbedGeom<LOG2M, LE>;
    if constexpr (S < G::SLOC || G::LOG2W == 0) {
        return t + (i << G::LOG2T);
    } else {
        return (t & 63) | (i << 6) | ((t >> 6) << (6 + G::log2I(S)));
    }
}

// Position (in the in-place layout) of element k of butterfly slot i of thread t at stage s.
template <int LOG2M, int LE, int S>
__device__ __forceinline__ int embed_pos(int t, int i, int k) {
    using G = EmbedGeom<LOG2M, LE>;
    constexpr int ls = G::log2S(S);
    constexpr int lb = ls + G::bits(S);
    const int b = embed_butterfly<LOG2M, LE, S>(t, i);
    const int blk = b >> ls;
    const int o = b & ((1 << ls) - 1);
    return (blk << lb) + o + (k << ls);
}


// Bank-conflict-avoiding permutation of positions inside one line: XOR the low bits of the
// position with bits of its higher digits. The bit choice was measured on gfx950 with the
// conflict counter over this kernel's exchange patterns (16-byte elements: bits 3 and 8 into the
// low 4 bits; 8-byte elements: bits 3 and 7 into the low 5 bits). The XOR stays inside an
// aligned group of at most M positions, so the permutation maps [0, M) onto itself.
template <typename T, int LOG2M>
__device__ __forceinline__ int embed_swz(int p) {
    constexpr bool wide = sizeof(cplx<T>) == 16;
    constexpr int A = 3, B = wide ? 8 : 7, W = wide ? 4 : 5;
    constexpr int bitsw = W < LOG2M ? W : LOG2M;
    constexpr int mask = (1 << bitsw) - 1;
    return p ^ (((p >> A) ^ (p >> B)) & mask);
}

// Twiddle of element k of slot i at stage s: W_M^{o k M / B_s}.
template <int LOG2M, int LE, int S>
__device__ __forceinline__ int embed_tw_index(int t, int i, int k) {
    using G = EmbedGeom<LOG2M, LE>;
    constexpr int ls = G::log2S(S);
    const int b = embed_butterfly<LOG2M, LE, S>(t, i);
    const int o = b & ((1 << ls) - 1);
    return (o * k) << G::log2Pre(S);
}

template <typename T, int LOG2M, int LE>
struct EmbedLine {
    using G = EmbedGeom<LOG2M, LE>;
    static constexpr int NTW = G::NST > 1 ? G::NST - 1 : 1;
    cplx<T> a[G::E];
    cplx<T> tw[NTW][G::E];

    __device__ __forceinline__ void load_twiddles(const cplx<T>* __restrict__ table, int t) {
        load_tw_stages(table, t, std::make_integer_sequence<int, G::NST - 1>{});
    }
    template <int... S>
    __device__ __forceinline__ void load_tw_stages(const cplx<T>* __restrict__ table, int t,
                                                   std::integer_sequence<int, S...>) {
        (load_tw_stage<S>(table, t), ...);
    }
    template <int S>
    __device__ __forceinline__ void load_tw_stage(const cplx<T>* __restrict__ table, int t) {
        constexpr int R = G::R(S);
#pragma unroll
        for (int i = 0; i < G::E / R; ++i) {
#pragma unroll
            for (int k = 1; k < R; ++k) tw[S][i * R + k] = table[embed_tw_index<LOG2M, LE, S>(t, i, k)];
        }
    }

    // forward radix pass S: DFT of every butterfly, then the pass twiddles (not after the last).
    // At pass 0 the inputs k >= R/2 sit at natural positions >= M/2 >= N: always zero.
    template <int S>
    __device__ __forceinline__ void fwd_stage() {
        constexpr int R = G::R(S);
#pragma unroll
        for (int i = 0; i < G::E / R; ++i) {
            if constexpr (S == 0 && R >= 2)
                dft_half_input<R, -1>(&a[i * R]);
            else
                dft<R, -1>(&a[i * R]);
            if constexpr (S < G::NST - 1) {
#pragma unroll
                for (int k = 1; k < R; ++k) a[i * R + k] = cmul(a[i * R + k], tw[S][i * R + k]);
            }
        }
    }
    // inverse radix pass S: conjugate twiddles, then the inverse DFT
    template <int S>
    __device__ __forceinline__ void inv_stage() {
        constexpr int R = G::R(S);
#pragma unroll
        for (int i = 0; i < G::E / R; ++i) {
            if constexpr (S < G::NST - 1) {
#pragma unroll
                for (int k = 1; k < R; ++k) a[i * R + k] = cmulc(a[i * R + k], tw[S][i * R + k]);
            }
            // at pass 0 the outputs k >= R/2 land at positions >= M/2 >= N and are discarded
            if constexpr (S == 0 && R >= 2)
                dft_half_output<R, +1>(&a[i * R]);
            else
                dft<R, +1>(&a[i * R]);
        }
    }

    // move the line's elements from the layout of pass SA to the layout of pass SB through LDS.
    // Between passes >= SLOC (or when a line fits in one wavefront) every wavefront writes and
    // then reads only positions whose top bits name it, so a wavefront-level ordering suffices;
    // the other exchanges cross wavefronts and take a workgroup barrier before the writes (no
    // wavefront may still be reading the positions) and between writes and reads.
    template <int SA, int SB>
    __device__ __forceinline__ void exchange(cplx<T>* __restrict__ line, int t) {
        constexpr int RA = G::R(SA), RB = G::R(SB);
        constexpr bool local = G::local(SA, SB);
        if constexpr (local)
            wave_sync();
        else
            __syncthreads();
#pragma unroll
        for (int i = 0; i < G::E / RA; ++i)
#pragma unroll
            for (int k = 0; k < RA; ++k) line[embed_swz<T, LOG2M>(embed_pos<LOG2M, LE, SA>(t, i, k))] = a[i * RA + k];
        if constexpr (local)
            wave_sync();
        else
            __syncthreads();
#pragma unroll
        for (int i = 0; i < G::E / RB; ++i)
#pragma unroll
            for (int k = 0; k < RB; ++k) a[i * RB + k] = line[embed_swz<T, LOG2M>(embed_pos<LOG2M, LE, SB>(t, i, k))];
        // issue all reads of the exchange back to back: one LDS latency per exchange instead of
        // one per element (the scheduler otherwise interleaves them with the arithmetic)
        __builtin_amdgcn_sched_barrier(0);
    }

    template <int S>
    __device__ __forceinline__ void fwd_from(cplx<T>* line, int t) {
        if constexpr (S > 0) exchange<S - 1, S>(line, t);
        fwd_stage<S>();
        if constexpr (S + 1 < G::NST) fwd_from<S + 1>(line, t);
    }
    template <int S>
    __device__ __forceinline__ void inv_from(cplx<T>* line, int t) {
        if constexpr (S < G::NST - 1) exchange<S + 1, S>(line, t);
        inv_stage<S>();
        if constexpr (S > 0) inv_from<S - 1>(line, t);
    }

    // multiply by the kernel spectrum, stored in last-pass position order: the spectrum values at
    // this thread's last-pass positions
    __device__ __forceinline__ void load_scale(const Spec<T>* __restrict__ g, Spec<T>* gv, int t) {
        constexpr int S = G::NST - 1;
        constexpr int R = G::R(S);
#pragma unroll
        for (int i = 0; i < G::E / R; ++i)
#pragma unroll
            for (int k = 0; k < R; ++k) gv[i * R + k] = g[embed_pos<LOG2M, LE, S>(t, i, k)];
    }
    __device__ __forceinline__ void scale(const Spec<T>* gv) {
#pragma unroll
        for (int e = 0; e < G::E; ++e) {
            a[e].x = spec_mul(a[e].x, gv[e]);
            a[e].y = spec_mul(a[e].y, gv[e]);
        }
    }

    // natural position of register (i, k) at pass 0
    static __device__ __forceinline__ int nat(int t, int i, int k) { return embed_pos<LOG2M, LE, 0>(t, i, k); }

    // one exponential factor: forward transform, spectrum, inverse transform, truncation; in the
    // increment form (FP32) the spectrum is that of the factor minus the identity and the
    // factor's input (the registers below M/2 at pass 0: the others hold zero padding) is kept
    // and added back
    __device__ __forceinline__ void factor(const Spec<T>* __restrict__ g, cplx<T>* line, int t, int n) {
        constexpr bool INC = increment_form<T>();
        constexpr int R0 = G::R(0);
        constexpr int H = R0 >= 2 ? R0 / 2 : 1;   // input registers per pass-0 butterfly
        cplx<T> x0[INC ? G::E / R0 * H : 1];
        if constexpr (INC) {
#pragma unroll
            for (int i = 0; i < G::E / R0; ++i)
#pragma unroll
                for (int k = 0; k < H; ++k) x0[i * H + k] = a[i * R0 + k];
        }
        // FP32 loads the spectrum after the forward transform: held across it, it would take the
        // kernels that also keep the input past 128 VGPRs; FP64 loads it first and hides the latency
        Spec<T> gv[G::E];
        if constexpr (!INC) load_scale(g, gv, t);
        fwd_from<0>(line, t);
        if constexpr (INC) load_scale(g, gv, t);
        scale(gv);
        inv_from<G::NST - 1>(line, t);
#pragma unroll
        for (int i = 0; i < G::E / R0; ++i)
#pragma unroll
            for (int k = 0; k < R0; ++k) {
                if (k >= R0 / 2 && R0 >= 2)
                    a[i * R0 + k] = {(T)0, (T)0};           // position >= M/2 >= N
                else if (nat(t, i, k) >= n)
                    a[i * R0 + k] = {(T)0, (T)0};
                else if constexpr (INC)
                    a[i * R0 + k] = a[i * R0 + k] + x0[i * H + k];
            }
    }
};

}  // namespace sfac
