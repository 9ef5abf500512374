// Host stand-ins for the kernel launch functions: every launch is validated (its state, tables and
// status words lie in live allocations; a grouped launch's descriptors are live and its block
// offsets consistent) when it runs, i.e. at once or, for a captured launch, at each graph replay.
#include <hip/hip_runtime.h>
#include <functional>
#include <cstdio>

#include "sfac_kernels.hpp"

[[noreturn]] void mock_die(const char* what);
bool mock_range_live(const void* p, size_t n);
void mock_submit(hipStream_t s, std::function<void()> f);
bool mock_inject();
hipError_t mock_fail_launch(hipStream_t s);

namespace sfac {

template <typename T>
int pass_blocks(const PassDesc<T>& d) {
    return d.xcd_remap ? 8 * ((d.ntiles + 7) / 8) : d.ntiles;
}

template <typename T>
static void check_desc(const PassDesc<T>& d) {
    const size_t n = (size_t)d.N * (size_t)d.inner * (size_t)d.outer;
    if (!mock_range_live(d.u, n * sizeof(T))) mock_die("pass reads a state outside live memory");
    if (!mock_range_live(d.stat_max, 8) || !mock_range_live(d.stat_flags, 4)) mock_die("status words not live");
    if (d.tw && !mock_range_live(d.tw, sizeof(cplx<T>))) mock_die("twiddles not live");
    if (d.gpos_c && !mock_range_live(d.gpos_c, sizeof(Spec<T>))) mock_die("spectrum table not live");
    if (d.ntiles <= 0 || d.lpb <= 0 || d.threads <= 0 || d.threads > 1024) mock_die("bad tile geometry");
}

template <typename T>
hipError_t launch_axis_pass(const PassDesc<T>& d, size_t lds, hipStream_t s) {
    if (lds > 160 * 1024) mock_die("LDS above 160 KiB");
    if (mock_inject()) return mock_fail_launch(s);
    const PassDesc<T> c = d;
    mock_submit(s, [c] { check_desc(c); });
    return hipSuccess;
}

template <typename T>
hipError_t launch_axis_pass_multi(int kind, int variant, int threads, const GroupArgs<T>& args, size_t lds,
                                  hipStream_t s) {
    if (args.n < 1 || args.n > kGroupSlots) mock_die("grouped launch with a bad instance count");
    if (threads < 1 || threads > 1024) mock_die("grouped launch with a bad block size");
    if (lds > 160 * 1024) mock_die("grouped launch above 160 KiB of LDS");
    (void)kind;
    (void)variant;
    if (mock_inject()) return mock_fail_launch(s);
    const GroupArgs<T> c = args;
    mock_submit(s, [c, threads] {
        for (int i = 0; i < c.n; ++i) {
            if (!mock_range_live(c.desc[i], sizeof(PassDesc<T>))) mock_die("grouped launch reads a freed descriptor");
            PassDesc<T> d = *c.desc[i];
            d.u = c.u[i];
            check_desc(d);
            if (c.start[i + 1] - c.start[i] != pass_blocks(d)) mock_die("block offsets disagree with the tiles");
            if (d.threads > threads) mock_die("block smaller than a descriptor's lines");
        }
    });
    return hipSuccess;
}

hipError_t launch_trace_collect(unsigned long long*, long long, unsigned long long*, long long*, long long,
                                hipStream_t s) {
    mock_submit(s, [] {});
    return hipSuccess;
}
hipError_t launch_exact_gemm(const double*, const double*, double*, int, int, int, long long, long long, long long,
                             long long, long long, long long, int, hipStream_t s) {
    mock_submit(s, [] {});
    return hipSuccess;
}
hipError_t launch_exact_nl(double*, const double*, long long, double, bool, int, const PassDesc<double>&, hipStream_t s) {
    mock_submit(s, [] {});
    return hipSuccess;
}
hipError_t launch_zero_words(unsigned int* p, int words, hipStream_t s) {
    if (words <= 0) return hipSuccess;
    if (!mock_range_live(p, sizeof(unsigned int) * (size_t)words)) mock_die("zero_words outside live memory");
    if (mock_inject()) return mock_fail_launch(s);
    mock_submit(s, [p, words] {
        if (!mock_range_live(p, sizeof(unsigned int) * (size_t)words)) mock_die("zero_words outside live memory");
        for (int i = 0; i < words; ++i) p[i] = 0u;
    });
    return hipSuccess;
}
hipError_t launch_timing_mark(int, hipStream_t s) {
    mock_submit(s, [] {});
    return hipSuccess;
}
template <typename T>
hipError_t launch_energy_pass(const PassDesc<T>&, size_t, hipStream_t s) {
    mock_submit(s, [] {});
    return hipSuccess;
}
template <typename T>
hipError_t allow_lds(size_t) {
    return hipSuccess;
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
