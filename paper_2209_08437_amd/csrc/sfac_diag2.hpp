// Register-resident axis pass for the diagonal method (Remark 1) when N = A * B with small
// coprime A, B.
//
// A length-N transform is done in two steps with the prime-factor (Good-Thomas) index maps, so
// no twiddles sit between them. Thread b (b < B) holds x[(B a + A b) mod N] for a < A and does
// one DFT of length A; after one LDS exchange thread k1 (k1 < A) holds the A-point results of
// all b and does one DFT of length B, which leaves X[(B (B^-1 mod A) k1 + A (A^-1 mod B) k2) mod N]
// in its registers k2. The inverse runs the conjugate steps in reverse order and returns every
// element to the thread and register that loaded it, exactly where the next forward transform
// reads it. Per factor: [psi multiply] forward transform, multiply by the eigenvalue factor,
// inverse transform, [conj(psi) multiply]: two LDS exchanges per factor, no padding.
// A line is held by P = max(A, B) threads; threads beyond A (or B) idle in the other step.
// Lines either follow each other across the block (the exchanges take workgroup barriers) or,
// in the wavefront-aligned layout, floor(64 / P) lines fill each wavefront and its remaining
// lanes idle (the exchanges stay inside one wavefront and need no workgroup barrier).
// Tables are stored per thread in the order the thread walks them (see the host builder).
#pragma once

#include <hip/hip_runtime.h>

#include "sfac_fft.hpp"

namespace sfac {

template <int A, int B>
struct Diag2Geom {
    static constexpr int N = A * B;
    static constexpr int P = A > B ? A : B;   // threads per line
    static constexpr int E = P;               // registers per thread (max of the two step sizes)
    static constexpr int LPW = 64 / P;        // lines per wavefront in the wavefront-aligned layout
    // natural position of register k of thread t (t < B, k < A)
    static __device__ __forceinline__ int pos(int t, int k) {
        const int n = B * k + A * t;
        return n < N ? n : n - N;
    }
};

template <typename T, int A, int B, bool WA>
struct Diag2Line {
    using G = Diag2Geom<A, B>;
    cplx<T> a[G::E];

    static __device__ __forceinline__ void sync() {
        if constexpr (WA)
            wave_sync();
        else
            __syncthreads();
    }

    // x <- psi . x (or conj(psi) . x) at this thread's natural positions;
    // psipos[t A + k] = psi at position pos(t, k)
    template <bool CONJ>
    __device__ __forceinline__ void psi_mul(const cplx<T>* __restrict__ psipos, int t) {
        if (t < B) {
#pragma unroll
            for (int k = 0; k < A; ++k) {
                const cplx<T> w = psipos[t * A + k];
                a[k] = CONJ ? cmulc(a[k], w) : cmul(a[k], w);
            }
        }
    }

    // forward: DFT_A in thread b, exchange, DFT_B in thread k1
    __device__ __forceinline__ void forward(cplx<T>* __restrict__ line, int t) {
        if (t < B) dft<A, -1>(a);
        sync();
        if (t < B) {
#pragma unroll
            for (int k = 0; k < A; ++k) line[k * B + t] = a[k];
        }
        sync();
        if (t < A) {
#pragma unroll
            for (int b = 0; b < B; ++b) a[b] = line[t * B + b];
            __builtin_amdgcn_sched_barrier(0);   // all reads in flight before the arithmetic
            dft<B, -1>(a);
        }
    }

    // inverse: conjugate DFT_B in thread k1, exchange, conjugate DFT_A in thread b
    __device__ __forceinline__ void inverse(cplx<T>* __restrict__ line, int t) {
        if (t < A) dft<B, +1>(a);
        sync();
        if (t < A) {
#pragma unroll
            for (int b = 0; b < B; ++b) line[t * B + b] = a[b];
        }
        sync();
        if (t < B) {
#pragma unroll
            for (int k = 0; k < A; ++k) a[k] = line[k * B + t];
            __builtin_amdgcn_sched_barrier(0);   // all reads in flight before the arithmetic
            dft<A, +1>(a);
        }
    }

    // eigenvalue factor of the frequency register k2 of thread k1 holds, stored as gpos[k1 B + k2]
    __device__ __forceinline__ void load_scale(const Spec<T>* __restrict__ gpos, Spec<T>* gv, int t) {
        if (t < A) {
#pragma unroll
            for (int b = 0; b < B; ++b) gv[b] = gpos[t * B + b];
        }
    }
    __device__ __forceinline__ void scale(const Spec<T>* gv, int t) {
        if (t < A) {
#pragma unroll
            for (int b = 0; b < B; ++b) {
                a[b].x = spec_mul(a[b].x, gv[b]);
                a[b].y = spec_mul(a[b].y, gv[b]);
            }
        }
    }

    // The eigenvalue factors are loaded after the forward transform, not before it: held across
    // the transform they would keep B more values live at its peak and cost the kernel a third
    // wavefront per SIMD (FP64 15 x 17: 202 against 156 VGPRs); their load latency is covered by
    // the other wavefronts that the smaller register budget lets in.
    // In the increment form (FP32) the tables hold the factor minus the identity and the factor's
    // input, kept in registers across it, is added back at the end.
    template <bool SKEW>
    __device__ __forceinline__ void factor(const Spec<T>* __restrict__ gpos, const cplx<T>* __restrict__ psipos,
                                           cplx<T>* line, int t) {
        constexpr bool INC = increment_form<T>();
        cplx<T> x0[INC ? A : 1];
        if constexpr (INC) {
#pragma unroll
            for (int k = 0; k < A; ++k) x0[k] = a[k];
        }
        if constexpr (SKEW) psi_mul<false>(psipos, t);
        forward(line, t);
        Spec<T> gv[B];
        load_scale(gpos, gv, t);
        scale(gv, t);
        inverse(line, t);
        if constexpr (SKEW) psi_mul<true>(psipos, t);
        if constexpr (INC) {
            if (t < B) {
#pragma unroll
                for (int k = 0; k < A; ++k) a[k] = a[k] + x0[k];
            }
        }
    }

    // the three factors e^{tau/2 C} e^{tau S} e^{tau/2 C}, the skew one wrapped in psi and conj(psi)
    __device__ __forceinline__ void factors(const Spec<T>* __restrict__ gpos_c, const Spec<T>* __restrict__ gpos_s,
                                            const cplx<T>* __restrict__ psipos, cplx<T>* line, int t) {
        factor<false>(gpos_c, psipos, line, t);
        factor<true>(gpos_s, psipos, line, t);
        factor<false>(gpos_c, psipos, line, t);
    }
};

}  // namespace sfac
