// Launch interface of the axis-pass kernels (host and device share these types).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sfac_fft.hpp"
#include "sfac_internal.hpp"

namespace sfac {

constexpr int kBlockThreads = 256;

// Block size bound of the embedded-method kernels whose tiles are staged through LDS, for lines
// of t threads: room for at least two line pairs, and at least 256 threads. (A larger bound
// would cut the register budget of the kernels with 16 elements per thread, which then spill.)
constexpr int embed_stage_block(int t) {
    return 2 * t > 1024 ? 1024 : (2 * t < 256 ? 256 : 2 * t);
}

// LDS elements per line of the two-step diagonal kernel (N = A B): N plus a pad that spreads
// the lanes of neighbouring lines over the banks; the pads come from a bank-conflict model of
// the kernel's access patterns (16-lane groups of 16-byte elements, 32-lane groups of 8-byte
// ones) at the usual lines per block.
constexpr int diag2_line_stride(int a, int b, int elem_bytes) {
    const int n = a * b;
    if (elem_bytes == 16) {
        if (a == 3 && b == 5) return n + 10;
        if (a == 5 && b == 7) return n + 10;
        if (a == 15 && b == 17) return n + 2;
    } else {
        if (a == 3 && b == 5) return n + 4;
        if (a == 5 && b == 7) return n + 7;
        if (a == 7 && b == 9) return n + 9;
        if (a == 9 && b == 11) return n + 4;
        if (a == 13 && b == 15) return n + 15;
    }
    return n;
}

// Everything one axis pass of one instance needs. Lines along the axis are addressed as
// u[o * N * inner + k * inner + i]: o < outer indexes the slower axes, i < inner the faster
// ones, k < N the position on the line. inner == 1 is the contiguous axis (axis 1).
template <typename T>
struct PassDesc {
    T* u;                            // state, device
    const cplx<T>* tw;               // e^{-2 pi i m / L}, m < L
    const Spec<T>* scale_c;          // diag: e^{tau/2 lambda}/N; embed: kernel spectrum / M
    const Spec<T>* scale_s;          // diag: e^{tau mu}/N;       embed: kernel spectrum / M
    const cplx<T>* psi;              // diag: e^{-i pi k / N}, k < N
    const Spec<T>* gpos_c;           // embed: kernel spectra / M in digit-reversed position order;
    const Spec<T>* gpos_s;           // two-step diagonal kernel: factors in per-thread order
    const cplx<T>* psi2;             // two-step diagonal kernel: per-thread psi
    unsigned long long* stat_max;    // bits of the largest |u| stored (non-negative double)
    unsigned int* stat_flags;        // SFAC_FLAG_* bits
    double* energy;                  // energy pass: [0] += sum of x^T B x over its lines, [1] += (u^2 - 1)^2 / 4
    unsigned long long* trace_part;  // last pass: one slot per wavefront (block b, wave w at b * trace_wpb + w)
    int trace_wpb;                   // for the largest |u| it stored (bits), or null when no record is kept
    long long inner, outer;
    int N;                           // points per line
    int L;                           // transform length (N or M)
    int method;                      // 1 diag, 2 embed
    int nst;                         // number of stages
    int radix[kMaxStages];
    int lpb;                         // complex lines (pairs of real lines) per block
    int tiles_per_outer;             // strided passes: ceil(inner / (2 lpb))
    int ntiles;                      // tiles in this pass
    int nl_in, nl_out;               // apply J^Q_{tau/2} on load / on store (+ statistics)
    int nl_mid;                      // the pass covers its axis twice, a step boundary between the two
                                     // (closing J^Q_{tau/2}, statistics, opening J^Q_{tau/2}, in registers)
    int xcd_remap;                   // group neighbouring tiles per XCD
    int d2wave;                      // two-step diagonal kernel: wavefront-aligned line layout
    int log2m;                       // embed: log2 of the transform length
    int log2e;                       // embed: log2 of the largest elements-per-thread count (2, 3 or 4)
    int stage;                       // embed: tile loaded and stored through LDS (coalesced walks)
    int d2a, d2b;                    // diag: N = d2a * d2b for the two-step kernel, 0 for the generic one
    int threads;                     // launch block size
    T decay, decay_lo;               // e^{-tau} = decay + decay_lo (decay_lo = 0 in FP64)
};

template <typename T>
int pass_blocks(const PassDesc<T>& d);

template <typename T>
hipError_t launch_axis_pass(const PassDesc<T>& d, size_t lds_bytes, hipStream_t stream);

// The instances of one grouped launch, passed by value as the kernel's argument (so a launch
// needs no device memory of its own and a captured graph node carries everything it reads):
// entry i is the device copy of a plan's pass descriptor (its `u` field unused), the state it
// steps, and its first block; start[n] is the launch's block count. A launch holds at most
// kGroupSlots instances (about 1.3 KB of kernel arguments); larger sets take several launches.
constexpr int kGroupSlots = 64;
constexpr int kTwiceVariant = 1 << 20;
template <typename T>
struct GroupArgs {
    const PassDesc<T>* desc[kGroupSlots];
    T* u[kGroupSlots];
    int start[kGroupSlots + 1];
    int n;
};

// One launch over several instances' tiles of one pass (or of two passes over one axis, when
// variant >= kTwiceVariant: descriptors with nl_mid); every descriptor of the launch uses the
// same kernel variant; `threads` is the block size (the group's largest).
// kind: 0 generic, 1 embedded (variant = log2m * 8 + log2e, plus 128 for the LDS-staged tile),
// 2 two-step diagonal (variant = a * 64 + b, plus 4096 for the wavefront-aligned line layout)
template <typename T>
hipError_t launch_axis_pass_multi(int kind, int variant, int threads, const GroupArgs<T>& args, size_t lds_bytes,
                                  hipStream_t stream);

// After the last pass of a step: reduce the nparts per-wavefront slots of the step's largest |u|
// into rec[*step] (if *step < cap), clear the slots and advance *step by one.
hipError_t launch_trace_collect(unsigned long long* parts, long long nparts, unsigned long long* rec, long long* step,
                                long long cap, hipStream_t stream);

// Clears `words` 32-bit words at p on `stream` with a kernel (not a memset node, so that a caller
// may capture the call into a graph and replay it).
hipError_t launch_zero_words(unsigned int* p, int words, hipStream_t stream);

// An empty kernel named for `axis` (1..3, or 0 after the last): sfac_plan_time_passes launches
// one before each axis' timed launches, so that profiles attribute those dispatches to their axis.
// Marker values: the axis (1..3) before the timed single-pass launches, kFusedMark + the axis
// before the timed launches that cover an axis twice, 0 after the last.
constexpr int kFusedMark = 10;
hipError_t launch_timing_mark(int axis, hipStream_t stream);

// The one-level scheme with the exact exponential (eq. (strang)), FP64.
// Batched row-major product C[b] = X[b] Y[b] (M x K times K x N; leading dimensions ldx, ldy, ldc
// and batch strides sx, sy, sc in elements; any sizes).
hipError_t launch_exact_gemm(const double* X, const double* Y, double* C, int M, int N, int K, long long ldx,
                             long long ldy, long long ldc, long long sx, long long sy, long long sc, int batch,
                             hipStream_t stream);
// dst[i] = J^Q_{tau/2}(src[i]) for i < n (dst may be src); with `stats`, the largest |u| and the
// non-finite flag are folded into d.stat_max / d.stat_flags (and d.trace_part) as by the last pass
// of the two-level scheme. `halves` = 2 applies the half-step twice, the statistics taken after
// the first (a step boundary: one step's closing half-step, the next one's opening), with the
// values of two launches of one half-step each. Blocks of 256 threads.
constexpr int kExactNlThreads = 256;
hipError_t launch_exact_nl(double* dst, const double* src, long long n, double decay, bool stats, int halves,
                           const PassDesc<double>& d, hipStream_t stream);

// Elements per thread (log2) of the energy kernel for a transform of length 2^log2m: 8, or 16 at
// M = 4096, so that a line is at most 256 threads.
constexpr int energy_log2e(int log2m) { return log2m >= 12 ? 4 : 3; }

// One axis of the discrete energy (Sec. 5, Example 5) of d.u: per line pair the length-M transform
// of the zero-padded pair, sum_m G[m] |X[m]|^2 with d.gpos_c = G (B's circulant embedding, 1/M folded
// in, last-pass position order) and d.tw the transform twiddles, added to d.energy[0]; with d.nl_in
// set, also (u^2 - 1)^2 / 4 over the loaded elements, added to d.energy[1]. d.L = M <= 4096.
template <typename T>
hipError_t launch_energy_pass(const PassDesc<T>& d, size_t lds_bytes, hipStream_t stream);

// Raise the dynamic-LDS limit of the pass kernels to lds_bytes (needed above 64 KiB).
template <typename T>
hipError_t allow_lds(size_t lds_bytes);

}  // namespace sfac
