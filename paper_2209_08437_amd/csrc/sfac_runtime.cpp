// C ABI of the library: plans, batches, the step loop (HIP graphs of captured launches),
// sticky status and error reporting. The arithmetic lives in the kernels (sfac_kernels.hip)
// and the FP64 host tables (sfac_tables.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <system_error>
#include <thread>
#include <type_traits>
#include <vector>

#include "sfac_embed.hpp"
#include "sfac_internal.hpp"
#include "sfac_kernels.hpp"

namespace {

thread_local std::string g_error;

sfac_status fail(sfac_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

sfac_status hip_fail(hipError_t e, const char* what) {
    return fail(SFAC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kLdsBudget = 64 * 1024;        // per block when more than one line fits
constexpr size_t kLdsMax = 160 * 1024;          // gfx950 LDS per CU

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Device copy of one axis' tables in the plan's arithmetic type.
struct AxisDevice {
    sfac::AxisTables host;
    size_t off_tw = 0, off_sc = 0, off_ss = 0, off_psi = 0, off_gc = 0, off_gs = 0, off_psi2 = 0;
    int lpb = 1;
    int threads = 256;
    int log2e = 4;
    int d2wave = 0;   // two-step diagonal kernel in the wavefront-aligned layout
    int stage = 0;    // embedded kernel with the tile staged through LDS
    size_t lds = 0;
};

template <typename T>
size_t axis_table_bytes(const sfac::AxisTables& t, size_t base, AxisDevice* ad) {
    size_t off = base;
    ad->off_tw = off;
    off = align_up(off + sizeof(sfac::cplx<T>) * t.length, 256);
    ad->off_sc = off;
    off = align_up(off + sizeof(sfac::Spec<T>) * t.scale_c.size(), 256);
    ad->off_ss = off;
    off = align_up(off + sizeof(sfac::Spec<T>) * t.scale_s.size(), 256);
    ad->off_psi = off;
    off = align_up(off + sizeof(sfac::cplx<T>) * t.psi_re.size(), 256);
    ad->off_gc = off;
    off = align_up(off + sizeof(sfac::Spec<T>) * t.gpos_c.size(), 256);
    ad->off_gs = off;
    off = align_up(off + sizeof(sfac::Spec<T>) * t.gpos_s.size(), 256);
    ad->off_psi2 = off;
    off = align_up(off + sizeof(sfac::cplx<T>) * t.psi2_re.size(), 256);
    return off;
}

template <typename T>
void axis_table_fill(const sfac::AxisTables& t, const AxisDevice& ad, unsigned char* host) {
    auto* tw = reinterpret_cast<sfac::cplx<T>*>(host + ad.off_tw);
    for (int m = 0; m < t.length; ++m) tw[m] = {(T)t.tw_re[m], (T)t.tw_im[m]};
    auto* sc = reinterpret_cast<sfac::Spec<T>*>(host + ad.off_sc);
    for (size_t m = 0; m < t.scale_c.size(); ++m) sc[m] = sfac::make_spec<T>(t.scale_c[m]);
    auto* ss = reinterpret_cast<sfac::Spec<T>*>(host + ad.off_ss);
    for (size_t m = 0; m < t.scale_s.size(); ++m) ss[m] = sfac::make_spec<T>(t.scale_s[m]);
    auto* ps = reinterpret_cast<sfac::cplx<T>*>(host + ad.off_psi);
    for (size_t m = 0; m < t.psi_re.size(); ++m) ps[m] = {(T)t.psi_re[m], (T)t.psi_im[m]};
    auto* gc = reinterpret_cast<sfac::Spec<T>*>(host + ad.off_gc);
    for (size_t m = 0; m < t.gpos_c.size(); ++m) gc[m] = sfac::make_spec<T>(t.gpos_c[m]);
    auto* gs = reinterpret_cast<sfac::Spec<T>*>(host + ad.off_gs);
    for (size_t m = 0; m < t.gpos_s.size(); ++m) gs[m] = sfac::make_spec<T>(t.gpos_s[m]);
    auto* psi2 = reinterpret_cast<sfac::cplx<T>*>(host + ad.off_psi2);
    for (size_t m = 0; m < t.psi2_re.size(); ++m) psi2[m] = {(T)t.psi2_re[m], (T)t.psi2_im[m]};
}

// One instance's geometry and tables: the part a plan and a batch entry share.
struct Instance {
    int dims = 0;
    int n[3] = {1, 1, 1};
    double alpha[3] = {0, 0, 0}, h[3] = {0, 0, 0};
    double eps = 0, tau = 0;
    sfac_dtype dt = SFAC_FP64;
    AxisDevice ax[3];
    size_t table_bytes = 0;   // tables only
    size_t lds_max = 0;
    long long points() const {
        long long p = 1;
        for (int a = 0; a < dims; ++a) p *= n[a];
        return p;
    }
};

sfac_status validate_instance(int dims, const int32_t* n, const double* alpha, double eps, double tau,
                              const double* h, const char* who) {
    if (dims < 1 || dims > 3) return fail(SFAC_EINVAL, "%sdims = %d, expected 1, 2 or 3", who, dims);
    if (!n || !alpha || !h) return fail(SFAC_EINVAL, "%sNULL n_axis, alpha_axis or h_axis", who);
    for (int a = 0; a < dims; ++a) {
        if (n[a] < 1) return fail(SFAC_EINVAL, "%sN_%d = %d, expected >= 1", who, a + 1, n[a]);
        if (!(alpha[a] > 1.0 && alpha[a] <= 2.0))
            return fail(SFAC_EINVAL, "%salpha_%d = %g is outside (1, 2]", who, a + 1, alpha[a]);
        if (!(h[a] > 0.0) || !std::isfinite(h[a]))
            return fail(SFAC_EINVAL, "%sh_%d = %g, expected finite > 0", who, a + 1, h[a]);
    }
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(SFAC_EINVAL, "%seps = %g, expected finite >= 0", who, eps);
    if (!(tau > 0.0) || !std::isfinite(tau)) return fail(SFAC_EINVAL, "%stau = %g, expected finite > 0", who, tau);
    long long pts = 1;
    for (int a = 0; a < dims; ++a) {
        pts *= n[a];
        if (pts > (1LL << 40)) return fail(SFAC_EINVAL, "%sgrid too large", who);
    }
    return SFAC_OK;
}

// Tables for every axis of one instance (host side); methods[a] may be AUTO.
sfac_status build_instance(Instance* in, int dims, const int32_t* n, const double* alpha, double eps,
                           double tau, const double* h, sfac_dtype dt, const sfac_options* opt,
                           const char* who) {
    const int32_t* methods = opt ? opt->method : nullptr;
    sfac_status st = validate_instance(dims, n, alpha, eps, tau, h, who);
    if (st != SFAC_OK) return st;
    in->dims = dims;
    in->eps = eps;
    in->tau = tau;
    in->dt = dt;
    const size_t elem = dt == SFAC_FP64 ? sizeof(sfac::cplx<double>) : sizeof(sfac::cplx<float>);
    size_t off = 0;
    for (int a = 0; a < dims; ++a) {
        in->n[a] = n[a];
        in->alpha[a] = alpha[a];
        in->h[a] = h[a];
        const int kern = opt ? opt->kernel[a] : 0;
        if (kern < 0 || kern > 4)
            return fail(SFAC_EINVAL, "%saxis %d: kernel = %d, expected 0 to 4", who, a + 1, kern);
        int m = methods ? methods[a] : SFAC_METHOD_AUTO;
        if (kern >= 1 && kern <= 3 && m == SFAC_METHOD_EMBED)
            return fail(SFAC_EINVAL, "%saxis %d: a diagonal-method kernel was chosen for the embedded method", who,
                        a + 1);
        if (kern == 4 && m == SFAC_METHOD_DIAG)
            return fail(SFAC_EINVAL, "%saxis %d: the staged embedded kernel was chosen for the diagonal method", who,
                        a + 1);
        if (m == SFAC_METHOD_AUTO)
            m = kern == 4 ? SFAC_METHOD_EMBED : (kern != 0 ? SFAC_METHOD_DIAG : sfac::auto_method(n[a], dt));
        if (m != SFAC_METHOD_DIAG && m != SFAC_METHOD_EMBED)
            return fail(SFAC_EUNSUPPORTED, "%saxis %d: no method supports N = %d", who, a + 1, n[a]);
        // embedded method: elements per thread. Fewer (8) doubles the threads of a line: worth it
        // when the pass would otherwise have too few waves to hide latency (under two per SIMD
        // of a 256-CU device); more (16) needs one radix pass less.
        int log2e = opt && opt->elems_log2[a] ? opt->elems_log2[a] : 0;
        if (log2e != 0 && log2e != 2 && log2e != 3 && log2e != 4)
            return fail(SFAC_EINVAL, "%saxis %d: elems_log2 = %d, expected 2, 3 or 4", who, a + 1, log2e);
        {
            long long inner0 = 1, outer0 = 1;
            for (int b = 0; b < a; ++b) inner0 *= n[b];
            for (int b = a + 1; b < dims; ++b) outer0 *= n[b];
            const long long avail0 = inner0 == 1 ? outer0 : inner0;
            const long long lines0 = outer0 * inner0 / avail0 * ((avail0 + 1) / 2);
            int mlen = sfac::embed_length(n[a]);
            if (log2e == 0) log2e = lines0 * (mlen / 16) / 64 < 2048 ? 3 : 4;
        }
        in->ax[a].log2e = log2e;
        sfac::AxisParams p{n[a], alpha[a], eps, tau, h[a]};
        std::string err = sfac::build_axis_tables(p, m, &in->ax[a].host, log2e, kern != 1,
                                                  dt == SFAC_FP32 /* FP32 kernels use the increment form */);
        if (!err.empty() && kern >= 2 && m == SFAC_METHOD_DIAG) err = "";
        if (kern >= 2 && m == SFAC_METHOD_DIAG && in->ax[a].host.d2a == 0)
            return fail(SFAC_EUNSUPPORTED, "%saxis %d: N = %d is not a product the register-resident diagonal "
                        "kernel handles", who, a + 1, n[a]);
        if (!err.empty()) {
            const bool range = err.find("exceeds") != std::string::npos || err.find("prime factor") != std::string::npos;
            return fail(range ? SFAC_EUNSUPPORTED : SFAC_EINVAL, "%saxis %d: %s", who, a + 1, err.c_str());
        }
        off = dt == SFAC_FP64 ? axis_table_bytes<double>(in->ax[a].host, off, &in->ax[a])
                              : axis_table_bytes<float>(in->ax[a].host, off, &in->ax[a]);
        const int L = in->ax[a].host.length;
        long long inner = 1, outer = 1;
        for (int b = 0; b < a; ++b) inner *= n[b];
        for (int b = a + 1; b < dims; ++b) outer *= n[b];
        const long long avail = (inner == 1 ? outer : inner);
        const long long lines_total = outer * inner / avail * ((avail + 1) / 2);
        if (m == SFAC_METHOD_EMBED) {
            // register-resident kernel: T = M/E threads per line, up to 256 threads per block;
            // fewer lines per block while that still leaves blocks for every CU
            int log2m = 0;
            while ((1 << log2m) < L) ++log2m;
            if (in->ax[a].log2e == 2 && (log2m < 6 || log2m > 11))
                return fail(SFAC_EUNSUPPORTED, "%saxis %d: elems_log2 = 2 needs a transform length of 64 to 2048, "
                            "not %d", who, a + 1, L);
            const int E = 1 << sfac::embed_log2e(log2m, in->ax[a].log2e);
            const int T = L / E;
            // staged tiles (kernel option 4): at least two lines per block, so that strided passes
            // read runs of several line pairs; otherwise 256 threads, or one line of 512 at E = 4
            const bool stage = kern == 4;
            if (stage && log2m < 6)
                return fail(SFAC_EUNSUPPORTED, "%saxis %d: staged tiles need a transform length of at least 64, "
                            "not %d", who, a + 1, L);
            const int max_block = stage ? sfac::embed_stage_block(T) : std::max(T, sfac::kBlockThreads);
            int lpb = max_block / T;
            const int keep = stage ? 2 : 1;
            while (lpb > keep && (lines_total + lpb - 1) / lpb < 1024) lpb >>= 1;
            if (opt && opt->lines_per_block[a] > 0) lpb = std::min(opt->lines_per_block[a], max_block / T);
            lpb = std::max(1, (int)std::min<long long>(lpb, std::max<long long>(1, (avail + 1) / 2)));
            in->ax[a].stage = stage ? 1 : 0;
            in->ax[a].lpb = lpb;
            in->ax[a].threads = lpb * T;
            in->ax[a].lds = elem * (size_t)L * lpb;
        } else if (in->ax[a].host.d2a > 0) {
            // two-step diagonal kernel: P = max(A, B) threads per line; by default at most 40 KB
            // of LDS lines per block, so that four blocks fit a CU
            const int P = std::max(in->ax[a].host.d2a, in->ax[a].host.d2b);
            const size_t ls = sfac::diag2_line_stride(in->ax[a].host.d2a, in->ax[a].host.d2b, (int)elem);
            const bool wave = kern == 3;
            const int lpw = 64 / P;   // lines per wavefront in the wavefront-aligned layout
            const int max_lines = wave ? (sfac::kBlockThreads / 64) * lpw : sfac::kBlockThreads / P;
            int lpb = std::min<int>(max_lines, std::max<size_t>(1, 40960 / (elem * ls)));
            if (wave) lpb = std::max(lpw, lpb / lpw * lpw);
            while (lpb > (wave ? lpw : 1) && (lines_total + lpb - 1) / lpb < 1024) lpb = wave ? lpb - lpw : lpb >> 1;
            if (opt && opt->lines_per_block[a] > 0) lpb = std::min(opt->lines_per_block[a], max_lines);
            lpb = std::max(1, (int)std::min<long long>(lpb, std::max<long long>(1, (avail + 1) / 2)));
            in->ax[a].lpb = lpb;
            in->ax[a].d2wave = wave ? 1 : 0;
            if (wave) {
                const int waves = (lpb + lpw - 1) / lpw;
                in->ax[a].threads = waves * 64;
                in->ax[a].lds = elem * ls * (size_t)(waves * lpw);   // every line slot of the block
            } else {
                in->ax[a].threads = lpb * P;
                in->ax[a].lds = elem * ls * lpb;
            }
        } else {
            // generic kernel: two LDS buffers per line (three in the increment form of FP32, which
            // keeps each factor's input), as many lines as fit the budget
            const size_t per_line = (dt == SFAC_FP32 ? 3 : 2) * elem * (size_t)L;
            int lpb = (int)std::max<size_t>(1, kLdsBudget / per_line);
            if (opt && opt->lines_per_block[a] > 0) lpb = opt->lines_per_block[a];
            lpb = (int)std::min<long long>(lpb, std::max<long long>(1, (avail + 1) / 2));
            lpb = std::min(lpb, 64);
            in->ax[a].lpb = lpb;
            in->ax[a].threads = sfac::kBlockThreads;
            in->ax[a].lds = per_line * lpb;
        }
        if (in->ax[a].lds > kLdsMax)
            return fail(SFAC_EUNSUPPORTED, "%saxis %d: transform length %d needs %zu bytes of LDS", who, a + 1, L,
                        in->ax[a].lds);
        in->lds_max = std::max(in->lds_max, in->ax[a].lds);
    }
    in->table_bytes = off;
    return SFAC_OK;
}

template <typename T>
sfac::PassDesc<T> make_desc(const Instance& in, int a, unsigned char* dev_tables, T* u,
                            unsigned long long* stat_max, unsigned int* stat_flags) {
    const AxisDevice& ad = in.ax[a];
    const sfac::AxisTables& t = ad.host;
    sfac::PassDesc<T> d{};
    d.u = u;
    d.tw = reinterpret_cast<const sfac::cplx<T>*>(dev_tables + ad.off_tw);
    d.scale_c = reinterpret_cast<const sfac::Spec<T>*>(dev_tables + ad.off_sc);
    d.scale_s = reinterpret_cast<const sfac::Spec<T>*>(dev_tables + ad.off_ss);
    d.psi = reinterpret_cast<const sfac::cplx<T>*>(dev_tables + ad.off_psi);
    d.gpos_c = reinterpret_cast<const sfac::Spec<T>*>(dev_tables + ad.off_gc);
    d.gpos_s = reinterpret_cast<const sfac::Spec<T>*>(dev_tables + ad.off_gs);
    d.threads = ad.threads;
    d.log2e = ad.log2e;
    d.d2a = t.d2a;
    d.d2b = t.d2b;
    d.d2wave = ad.d2wave;
    d.stage = ad.stage;
    d.psi2 = reinterpret_cast<const sfac::cplx<T>*>(dev_tables + ad.off_psi2);
    d.log2m = 0;
    while ((1 << d.log2m) < t.length) ++d.log2m;
    d.stat_max = stat_max;
    d.stat_flags = stat_flags;
    long long inner = 1, outer = 1;
    for (int b = 0; b < a; ++b) inner *= in.n[b];
    for (int b = a + 1; b < in.dims; ++b) outer *= in.n[b];
    d.inner = inner;
    d.outer = outer;
    d.N = t.n;
    d.L = t.length;
    d.method = t.method;
    d.nst = (int)t.radices.size();
    for (int s = 0; s < d.nst; ++s) d.radix[s] = t.radices[s];
    d.lpb = ad.lpb;
    if (inner == 1) {
        d.tiles_per_outer = 0;
        d.ntiles = (int)((outer + 2LL * d.lpb - 1) / (2LL * d.lpb));
    } else {
        d.tiles_per_outer = (int)((inner + 2LL * d.lpb - 1) / (2LL * d.lpb));
        d.ntiles = (int)(outer * d.tiles_per_outer);
    }
    d.nl_in = a == 0;
    d.nl_out = a == in.dims - 1;
    d.xcd_remap = inner > 1 ? 1 : 0;
    const double decay = std::exp(-in.tau);
    d.decay = (T)decay;
    d.decay_lo = (T)(decay - (double)d.decay);
    return d;
}

template <typename T>
hipError_t launch_pass(const sfac::PassDesc<T>& d, size_t lds, hipStream_t s) {
    return sfac::launch_axis_pass<T>(d, lds, s);
}

// The descriptor of axis a in a step that runs the axes in reverse order (d..1): the opening
// half-step moves to the pass of the last axis, the closing one (with the statistics) to the
// pass of the first. The factors of different axes commute (C_a and S_a are Kronecker sums), so
// every order applies the same operator; steps alternate between the two orders with the
// parity of the step count, which puts two passes over one axis next to each other at every
// step boundary.
template <typename T>
sfac::PassDesc<T> reversed_desc(sfac::PassDesc<T> d, int a, int dims) {
    d.nl_in = a == dims - 1;
    d.nl_out = a == 0;
    return d;
}

// Kernels that cover their axis twice in one launch (nl_mid) with values bitwise those of two
// launches, as measured against two launches for every transform length up to 2048 and every
// elements-per-thread choice: the two-step diagonal ones and the embedded ones. Lengths above
// 2048 (not measured) keep one launch per pass, as does the generic kernel.
template <typename T>
bool can_fuse(const sfac::PassDesc<T>& d) {
    if (d.method == SFAC_METHOD_DIAG) return d.d2a > 0;
    return d.method == SFAC_METHOD_EMBED && d.log2m <= 11;
}

// The launch that covers axis a twice: the last pass of a step (`cur`, from the step's
// descriptors) and the first pass of the next step (`next`, from the other order's).
template <typename T>
sfac::PassDesc<T> fused_desc(const sfac::PassDesc<T>& cur, const sfac::PassDesc<T>& next) {
    sfac::PassDesc<T> x = cur;
    x.nl_mid = 1;
    x.nl_out = next.nl_out;   // one axis: the next step's pass is also its last
    return x;
}

// Launches `nsteps` steps from step parity `parity0` (even: axes 1..d; odd: d..1), the passes
// of axis a taking fwd[a] or rev[a]. With `fuse`, the last pass of a step and the first of the
// next (the same axis) are one launch that covers the axis twice, the step boundary applied in
// registers: the state makes one trip through HBM instead of two and the values are bitwise
// those of the two launches. `after_step` (or null) runs after each step's last launch.
template <typename T, typename AfterStep>
hipError_t launch_sequence(const sfac::PassDesc<T>* fwd, const sfac::PassDesc<T>* rev, const Instance& in,
                           int parity0, int64_t nsteps, bool fuse, hipStream_t s, AfterStep after_step) {
    const int dims = in.dims;
    bool carried = false;   // this step's first pass was done by the previous launch
    for (int64_t k = 0; k < nsteps; ++k) {
        const bool odd = ((parity0 + k) & 1) != 0;
        const sfac::PassDesc<T>* D = odd ? rev : fwd;
        const sfac::PassDesc<T>* next = odd ? fwd : rev;
        for (int pos = 0; pos < dims; ++pos) {
            const int a = odd ? dims - 1 - pos : pos;
            if (pos == 0 && carried) {
                carried = false;
                continue;
            }
            sfac::PassDesc<T> x = D[a];
            if (pos == dims - 1 && fuse && k + 1 < nsteps && can_fuse(x)) {
                x = fused_desc(x, next[a]);
                carried = true;
            }
            const hipError_t e = launch_pass(x, in.ax[a].lds, s);
            if (e != hipSuccess) return e;
        }
        const hipError_t e = after_step(s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

// ===================================================================== plans
// Energy kernel of one axis (built on the first sfac_plan_energy call of a plan).
struct EnergyAxis {
    size_t off_tw = 0, off_g = 0;
    int log2m = 0, lpb = 1, threads = 64;
    size_t lds = 0;
};

namespace {
// A captured sequence of `steps` whole steps of a plan, replayed by sfac_step.
struct StepGraph {
    int64_t steps;
    int parity;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

std::atomic<unsigned long long> g_next_plan_id{1};
}  // namespace

struct sfac_plan_s {
    Instance in;
    unsigned long long id = g_next_plan_id.fetch_add(1);   // never reused (groups key graphs by it)
    hipStream_t stream = nullptr;      // caller's stream (may be the legacy default stream)
    hipStream_t capture = nullptr;     // private stream used only to capture graphs
    unsigned char* dev = nullptr;      // tables, status words, pass descriptors
    size_t dev_bytes = 0;
    size_t off_stat = 0;
    size_t off_desc = 0;               // device copies of d64 (FP64) or d32 (FP32), state pointer unset
    sfac::PassDesc<double> d64[3];     // axes in the order 1..d (even steps)
    sfac::PassDesc<float> d32[3];
    sfac::PassDesc<double> r64[3];     // axes in the order d..1 (odd steps)
    sfac::PassDesc<float> r32[3];
    int parity = 0;                    // parity of the steps queued so far (the next step's axis order)
    int use_graph = 1;
    int chunk = 32;
    void* graph_u = nullptr;           // state pointer the graphs were captured for
    // graphs of `chunk` steps and of powers of two below it, per starting parity, each captured
    // on first use
    std::vector<StepGraph> graphs;
    unsigned char* energy_dev = nullptr;  // [0, 16): the two energy sums; then per-axis tables
    size_t energy_bytes = 0;
    EnergyAxis eax[3];
    // per-step record: [0, 8) the step index, then trace_cap entries, then one slot per
    // wavefront of the last pass
    unsigned char* trace_dev = nullptr;
    long long trace_cap = 0, trace_parts = 0;
    int trace_wpb_last = 0, trace_wpb_first = 0;   // wavefronts per block of the passes of axis d and axis 1
    // one-level scheme with the exact exponential (SFAC_METHOD_EXACT): e^{tau B} per axis and a
    // state-sized scratch buffer in dev
    int exact = 0;
    size_t off_P[3] = {0, 0, 0}, off_scratch = 0;

    long long* trace_step() { return reinterpret_cast<long long*>(trace_dev); }
    unsigned long long* trace_rec() { return reinterpret_cast<unsigned long long*>(trace_dev + 8); }
    unsigned long long* trace_slots() { return trace_rec() + trace_cap; }
    void set_trace() {
        for (int a = 0; a < in.dims; ++a) {
            d64[a].trace_part = d32[a].trace_part = r64[a].trace_part = r32[a].trace_part = nullptr;
            d64[a].trace_wpb = d32[a].trace_wpb = r64[a].trace_wpb = r32[a].trace_wpb = 0;
        }
        if (trace_dev) {
            // the passes that store (and fold) the statistics: the last axis in even steps, the
            // first in odd ones
            const int a = in.dims - 1;
            d64[a].trace_part = d32[a].trace_part = r64[0].trace_part = r32[0].trace_part = trace_slots();
            d64[a].trace_wpb = d32[a].trace_wpb = trace_wpb_last;
            r64[0].trace_wpb = r32[0].trace_wpb = trace_wpb_first;
        }
    }

    unsigned long long* stat_max() { return reinterpret_cast<unsigned long long*>(dev + off_stat); }
    unsigned int* stat_flags() { return reinterpret_cast<unsigned int*>(dev + off_stat + 8); }

    void drop_graphs() {
        for (auto& sg : graphs) {
            (void)hipGraphExecDestroy(sg.exec);
            (void)hipGraphDestroy(sg.graph);
        }
        graphs.clear();
        graph_u = nullptr;
    }

    // device copy of axis a's descriptor for steps in the order 1..d (rev = 0) or d..1 (rev = 1)
    template <typename T>
    const sfac::PassDesc<T>* device_desc(int a, int rev) const {
        return reinterpret_cast<const sfac::PassDesc<T>*>(dev + off_desc) + 3 * rev + a;
    }
    // device copy of the descriptor of two passes in one launch: over axis 1 after a step in the
    // order d..1 (which = 0), over axis d after a step in the order 1..d (which = 1)
    template <typename T>
    const sfac::PassDesc<T>* fused_device_desc(int which) const {
        return reinterpret_cast<const sfac::PassDesc<T>*>(dev + off_desc) + 6 + which;
    }

    // eq. (strang): J^Q_{tau/2} e^{tau A} J^Q_{tau/2}, e^{tau A} one dense product per axis, alternating
    // between the state and the scratch buffer; the closing half-step writes the state and the
    // statistics of `stats`. With `ev` (2 per axis), each product is bracketed by an event pair.
    // Within a run of steps the closing launch of one step also applies the next one's opening
    // half-step (`open` false for that next step, `chain` true for this one), with the values of
    // separate launches.
    hipError_t exact_step(hipStream_t s, const sfac::PassDesc<double>& stats, hipEvent_t* ev = nullptr,
                          bool open = true, bool chain = false) {
        double* u = d64[0].u;
        double* scratch = reinterpret_cast<double*>(dev + off_scratch);
        const long long pts = in.points();
        const double decay = std::exp(-in.tau);
        hipError_t e = open ? sfac::launch_exact_nl(u, u, pts, decay, false, 1, stats, s) : hipSuccess;
        double* cur = u;
        double* other = scratch;
        for (int a = 0; a < in.dims && e == hipSuccess; ++a) {
            const long long n = in.n[a];
            long long inner = 1, outer = 1;
            for (int b = 0; b < a; ++b) inner *= in.n[b];
            for (int b = a + 1; b < in.dims; ++b) outer *= in.n[b];
            const double* P = reinterpret_cast<const double*>(dev + off_P[a]);
            if (ev) e = hipEventRecord(ev[2 * a], s);
            if (e != hipSuccess) break;
            if (inner == 1)   // rows: C = X P (P symmetric)
                e = sfac::launch_exact_gemm(cur, P, other, (int)outer, (int)n, (int)n, n, n, n, 0, 0, 0, 1, s);
            else              // per slower index o: C_o = P X_o
                e = sfac::launch_exact_gemm(P, cur, other, (int)n, (int)inner, (int)n, n, inner, inner, 0,
                                            n * inner, n * inner, (int)outer, s);
            if (ev && e == hipSuccess) e = hipEventRecord(ev[2 * a + 1], s);
            std::swap(cur, other);
        }
        if (e == hipSuccess) e = sfac::launch_exact_nl(u, cur, pts, decay, true, chain ? 2 : 1, stats, s);
        return e;
    }

    // `nsteps` steps from step parity `parity0`. The per-step record is folded after every step:
    // with two or more axes a fused launch stores the statistics of the step it closes (its
    // second pass opens the next step and closes none); with one axis both of its passes close a
    // step, so a plan of one axis that keeps the record does not fuse (the values are the same
    // either way).
    hipError_t launch_steps(hipStream_t s, int64_t nsteps, int parity0) {
        auto collect = [this](hipStream_t st) -> hipError_t {
            return trace_dev ? sfac::launch_trace_collect(trace_slots(), trace_parts, trace_rec(), trace_step(),
                                                          trace_cap, st)
                             : hipSuccess;
        };
        if (exact) {
            for (int64_t k = 0; k < nsteps; ++k) {
                hipError_t e = exact_step(s, d64[in.dims - 1], nullptr, k == 0, k + 1 < nsteps);
                if (e == hipSuccess) e = collect(s);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        }
        const bool fuse = trace_dev == nullptr || in.dims >= 2;
        return in.dt == SFAC_FP64 ? launch_sequence(d64, r64, in, parity0, nsteps, fuse, s, collect)
                                  : launch_sequence(d32, r32, in, parity0, nsteps, fuse, s, collect);
    }

    void set_u(void* u) {
        for (int a = 0; a < in.dims; ++a) {
            d64[a].u = r64[a].u = static_cast<double*>(u);
            d32[a].u = r32[a].u = static_cast<float*>(u);
        }
    }

    // the private capture stream, created on first use (plans stepped only through groups, or
    // with plain launches, never hold one)
    hipError_t capture_stream() {
        return capture ? hipSuccess : hipStreamCreateWithFlags(&capture, hipStreamNonBlocking);
    }

    sfac_status capture_graph(int64_t steps, int parity0, hipGraph_t* g, hipGraphExec_t* x) {
        *g = nullptr;
        *x = nullptr;
        hipError_t e = capture_stream();
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
        e = hipStreamBeginCapture(capture, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        hipError_t le = launch_steps(capture, steps, parity0);
        e = hipStreamEndCapture(capture, g);
        if (le != hipSuccess || e != hipSuccess) {
            if (e == hipSuccess && *g) (void)hipGraphDestroy(*g);
            *g = nullptr;
            return le != hipSuccess ? hip_fail(le, "kernel launch during capture") : hip_fail(e, "hipStreamEndCapture");
        }
        e = hipGraphInstantiate(x, *g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(*g);
            *g = nullptr;
            *x = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
        return SFAC_OK;
    }

    // the graph of `steps` steps from step parity `parity0` for the current state pointer,
    // captured on first use
    sfac_status graph_for(int64_t steps, int parity0, hipGraphExec_t* x) {
        for (const auto& sg : graphs)
            if (sg.steps == steps && sg.parity == parity0) {
                *x = sg.exec;
                return SFAC_OK;
            }
        StepGraph sg{steps, parity0, nullptr, nullptr};
        const sfac_status st = capture_graph(steps, parity0, &sg.graph, &sg.exec);
        if (st != SFAC_OK) return st;
        graphs.push_back(sg);
        *x = sg.exec;
        return SFAC_OK;
    }
};

namespace {

template <typename T>
sfac::PassDesc<T> energy_desc(const Instance& in, int a, const EnergyAxis& ea, unsigned char* dev, T* u) {
    sfac::PassDesc<T> d{};
    d.u = u;
    d.tw = reinterpret_cast<const sfac::cplx<T>*>(dev + ea.off_tw);
    d.gpos_c = reinterpret_cast<const sfac::Spec<T>*>(dev + ea.off_g);
    d.energy = reinterpret_cast<double*>(dev);
    d.log2m = ea.log2m;
    d.log2e = sfac::energy_log2e(ea.log2m);
    d.threads = ea.threads;
    long long inner = 1, outer = 1;
    for (int b = 0; b < a; ++b) inner *= in.n[b];
    for (int b = a + 1; b < in.dims; ++b) outer *= in.n[b];
    d.inner = inner;
    d.outer = outer;
    d.N = in.n[a];
    d.L = 1 << ea.log2m;
    d.method = SFAC_METHOD_EMBED;
    d.lpb = ea.lpb;
    if (inner == 1) {
        d.tiles_per_outer = 0;
        d.ntiles = (int)((outer + 2LL * d.lpb - 1) / (2LL * d.lpb));
    } else {
        d.tiles_per_outer = (int)((inner + 2LL * d.lpb - 1) / (2LL * d.lpb));
        d.ntiles = (int)(outer * d.tiles_per_outer);
    }
    d.nl_in = a == 0;
    d.xcd_remap = inner > 1 ? 1 : 0;
    return d;
}

// Host tables of every axis' energy kernel, uploaded once into a buffer of the plan.
template <typename T>
sfac_status energy_setup(sfac_plan p) {
    std::vector<unsigned char> host(256, 0);
    size_t lds_max = 0;
    for (int a = 0; a < p->in.dims; ++a) {
        const sfac::AxisParams ap{p->in.n[a], p->in.alpha[a], p->in.eps, p->in.tau, p->in.h[a]};
        sfac::EnergyTables t;
        int log2m = 0;
        while ((1 << log2m) < sfac::embed_length(p->in.n[a])) ++log2m;
        const std::string err = sfac::build_energy_tables(ap, sfac::energy_log2e(log2m), &t);
        if (!err.empty()) return fail(SFAC_EUNSUPPORTED, "energy, axis %d: %s", a + 1, err.c_str());
        EnergyAxis& ea = p->eax[a];
        ea.log2m = log2m;
        const int M = t.length;
        const int tl = M >> sfac::embed_log2e(log2m, sfac::energy_log2e(log2m));   // threads per line
        long long inner = 1, outer = 1;
        for (int b = 0; b < a; ++b) inner *= p->in.n[b];
        for (int b = a + 1; b < p->in.dims; ++b) outer *= p->in.n[b];
        const long long avail = inner == 1 ? outer : inner;
        ea.lpb = (int)std::max<long long>(1, std::min<long long>(std::max(1, sfac::kBlockThreads / tl),
                                                                 (avail + 1) / 2));
        ea.threads = ea.lpb * tl;
        ea.lds = sizeof(sfac::cplx<T>) * (size_t)M * ea.lpb;
        lds_max = std::max(lds_max, ea.lds);
        ea.off_tw = align_up(host.size(), 256);
        host.resize(ea.off_tw + sizeof(sfac::cplx<T>) * M);
        auto* tw = reinterpret_cast<sfac::cplx<T>*>(host.data() + ea.off_tw);
        for (int m = 0; m < M; ++m) tw[m] = {(T)t.tw_re[m], (T)t.tw_im[m]};
        ea.off_g = align_up(host.size(), 256);
        host.resize(ea.off_g + sizeof(sfac::Spec<T>) * M);
        auto* g = reinterpret_cast<sfac::Spec<T>*>(host.data() + ea.off_g);
        for (int m = 0; m < M; ++m) g[m] = sfac::make_spec<T>(t.gpos[m]);
    }
    unsigned char* dev = nullptr;
    hipError_t e = hipMalloc(&dev, host.size());
    if (e != hipSuccess)
        return e == hipErrorOutOfMemory ? fail(SFAC_ENOMEM, "hipMalloc(%zu): %s", host.size(), hipGetErrorString(e))
                                        : hip_fail(e, "hipMalloc");
    e = hipMemcpy(dev, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && lds_max > 64 * 1024) e = sfac::allow_lds<T>(lds_max);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return hip_fail(e, "energy tables");
    }
    p->energy_dev = dev;
    p->energy_bytes = host.size();
    return SFAC_OK;
}

template <typename T>
hipError_t energy_launch(sfac_plan p, T* u) {
    hipError_t e = sfac::launch_zero_words(reinterpret_cast<unsigned int*>(p->energy_dev), 4, p->stream);
    for (int a = 0; a < p->in.dims && e == hipSuccess; ++a)
        e = sfac::launch_energy_pass<T>(energy_desc<T>(p->in, a, p->eax[a], p->energy_dev, u), p->eax[a].lds,
                                        p->stream);
    return e;
}

}  // namespace

extern "C" {

const char* sfac_last_error(void) { return g_error.c_str(); }

}  // extern "C"

// A plan of the one-level scheme with the exact exponential: every axis SFAC_METHOD_EXACT, FP64.
static sfac_status exact_plan_create(sfac_plan p, int32_t dims, const int32_t* n, const double* alpha, double eps,
                                     double tau, const double* h, sfac_dtype dt, void* hip_stream,
                                     const sfac_options* opt) {
    sfac_status st = validate_instance(dims, n, alpha, eps, tau, h, "");
    if (st != SFAC_OK) return st;
    for (int a = 0; a < dims; ++a)
        if (opt->method[a] != SFAC_METHOD_EXACT)
            return fail(SFAC_EINVAL, "axis %d: the exact exponential replaces the whole linear step, so every axis "
                        "must use SFAC_METHOD_EXACT", a + 1);
    if (dt != SFAC_FP64) return fail(SFAC_EUNSUPPORTED, "the exact exponential is FP64 only");
    Instance& in = p->in;
    in.dims = dims;
    in.eps = eps;
    in.tau = tau;
    in.dt = dt;
    // e^{tau B} per axis: an axis with the same (N, alpha, h) as an earlier one reuses its matrix;
    // the others are built on threads of their own (each an O(N^3) eigendecomposition)
    std::vector<std::vector<double>> P(dims);
    std::vector<std::string> errs(dims);
    int same[3] = {-1, -1, -1};
    for (int a = 0; a < dims; ++a)
        for (int b = 0; b < a && same[a] < 0; ++b)
            if (same[b] < 0 && n[b] == n[a] && alpha[b] == alpha[a] && h[b] == h[a]) same[a] = b;
    auto build = [&](int a) {
        try {
            errs[a] = sfac::build_exact_exponential(sfac::AxisParams{n[a], alpha[a], eps, tau, h[a]}, &P[a]);
        } catch (const std::bad_alloc&) {
            errs[a] = "host allocation failed";
        }
    };
    std::vector<std::thread> workers;
    for (int a = 1; a < dims; ++a) {
        if (same[a] >= 0) continue;
        try {
            workers.emplace_back(build, a);
        } catch (const std::system_error&) {
            build(a);   // no thread to be had: build it here
        }
    }
    build(0);
    for (auto& w : workers) w.join();
    size_t off = 0;
    for (int a = 0; a < dims; ++a) {
        in.n[a] = n[a];
        in.alpha[a] = alpha[a];
        in.h[a] = h[a];
        if (same[a] >= 0) {
            p->off_P[a] = p->off_P[same[a]];
            continue;
        }
        if (!errs[a].empty()) return fail(SFAC_EUNSUPPORTED, "axis %d: %s", a + 1, errs[a].c_str());
        p->off_P[a] = off;
        off = align_up(off + sizeof(double) * P[a].size(), 256);
    }
    p->exact = 1;
    p->off_scratch = off;
    p->off_stat = align_up(off + sizeof(double) * (size_t)in.points(), 256);
    p->dev_bytes = p->off_stat + 256;
    p->stream = static_cast<hipStream_t>(hip_stream);
    p->use_graph = opt->use_graph ? 1 : 0;
    if (opt->graph_chunk > 0) p->chunk = opt->graph_chunk;
    std::vector<unsigned char> host(off, 0);
    for (int a = 0; a < dims; ++a)
        if (same[a] < 0) memcpy(host.data() + p->off_P[a], P[a].data(), sizeof(double) * P[a].size());
    hipError_t e = hipMalloc(&p->dev, p->dev_bytes);
    if (e != hipSuccess) {
        p->dev = nullptr;
        return e == hipErrorOutOfMemory ? fail(SFAC_ENOMEM, "hipMalloc(%zu): %s", p->dev_bytes, hipGetErrorString(e))
                                        : hip_fail(e, "hipMalloc");
    }
    e = hipMemcpy(p->dev, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(p->dev + p->off_stat, 0, 256);
    if (e != hipSuccess) {
        (void)hipFree(p->dev);
        p->dev = nullptr;
        return hip_fail(e, "exact plan set-up");
    }
    for (int a = 0; a < dims; ++a) {
        p->d64[a] = sfac::PassDesc<double>{};
        p->d64[a].stat_max = p->stat_max();
        p->d64[a].stat_flags = p->stat_flags();
    }
    return SFAC_OK;
}

extern "C" {

sfac_status sfac_plan_create(sfac_plan* out, int32_t dims, const int32_t* n_axis, const double* alpha_axis,
                             double eps, double tau, const double* h_axis, sfac_dtype dt, void* hip_stream,
                             const sfac_options* opt) {
    g_error.clear();
    if (!out) return fail(SFAC_EINVAL, "NULL output handle");
    *out = nullptr;
    if (dt != SFAC_FP64 && dt != SFAC_FP32) return fail(SFAC_EINVAL, "unknown dtype %d", (int)dt);
    if (opt) {
        if (opt->graph_chunk < 0 || opt->graph_chunk > 1024)
            return fail(SFAC_EINVAL, "graph_chunk = %d, expected 1..1024 (0 = default)", opt->graph_chunk);
        for (int a = 0; a < 3; ++a) {
            if (opt->method[a] < SFAC_METHOD_AUTO || opt->method[a] > SFAC_METHOD_EXACT)
                return fail(SFAC_EINVAL, "unknown method %d for axis %d", opt->method[a], a + 1);
            if (opt->lines_per_block[a] < 0 || opt->lines_per_block[a] > 256)
                return fail(SFAC_EINVAL, "lines_per_block = %d for axis %d, expected 0..256",
                            opt->lines_per_block[a], a + 1);
        }
    }
    std::unique_ptr<sfac_plan_s> p(new (std::nothrow) sfac_plan_s());
    if (!p) return fail(SFAC_ENOMEM, "host allocation failed");
    bool exact = false;
    for (int a = 0; opt && a < dims && a < 3; ++a) exact = exact || opt->method[a] == SFAC_METHOD_EXACT;
    if (exact) {
        sfac_status st = exact_plan_create(p.get(), dims, n_axis, alpha_axis, eps, tau, h_axis, dt, hip_stream, opt);
        if (st != SFAC_OK) return st;
        *out = p.release();
        return SFAC_OK;
    }
    sfac_status st = build_instance(&p->in, dims, n_axis, alpha_axis, eps, tau, h_axis, dt, opt, "");
    if (st != SFAC_OK) return st;
    p->stream = static_cast<hipStream_t>(hip_stream);
    if (opt) {
        p->use_graph = opt->use_graph ? 1 : 0;
        if (opt->graph_chunk > 0) p->chunk = opt->graph_chunk;
    }
    p->off_stat = align_up(p->in.table_bytes, 256);
    p->off_desc = p->off_stat + 256;
    const size_t desc_bytes = dt == SFAC_FP64 ? sizeof(sfac::PassDesc<double>) : sizeof(sfac::PassDesc<float>);
    p->dev_bytes = align_up(p->off_desc + 8 * desc_bytes, 256);   // three axes, two orders; two fused
    std::vector<unsigned char> host(p->dev_bytes, 0);
    for (int a = 0; a < p->in.dims; ++a) {
        if (dt == SFAC_FP64)
            axis_table_fill<double>(p->in.ax[a].host, p->in.ax[a], host.data());
        else
            axis_table_fill<float>(p->in.ax[a].host, p->in.ax[a], host.data());
    }
    hipError_t e = hipMalloc(&p->dev, p->dev_bytes);
    if (e != hipSuccess) {
        p->dev = nullptr;
        return e == hipErrorOutOfMemory ? fail(SFAC_ENOMEM, "hipMalloc(%zu): %s", p->dev_bytes, hipGetErrorString(e))
                                        : hip_fail(e, "hipMalloc");
    }
    for (int a = 0; a < p->in.dims; ++a) {
        p->d64[a] = make_desc<double>(p->in, a, p->dev, nullptr, p->stat_max(), p->stat_flags());
        p->d32[a] = make_desc<float>(p->in, a, p->dev, nullptr, p->stat_max(), p->stat_flags());
        p->r64[a] = reversed_desc(p->d64[a], a, p->in.dims);
        p->r32[a] = reversed_desc(p->d32[a], a, p->in.dims);
    }
    // the descriptors grouped launches read (the state pointer comes with each launch): the
    // three axes in the order 1..d, three in the order d..1, then the two fused launches
    const int dl = p->in.dims - 1;
    if (dt == SFAC_FP64) {
        const sfac::PassDesc<double> f[2] = {fused_desc(p->r64[0], p->d64[0]), fused_desc(p->d64[dl], p->r64[dl])};
        memcpy(host.data() + p->off_desc, p->d64, sizeof(sfac::PassDesc<double>) * p->in.dims);
        memcpy(host.data() + p->off_desc + 3 * desc_bytes, p->r64, sizeof(sfac::PassDesc<double>) * p->in.dims);
        memcpy(host.data() + p->off_desc + 6 * desc_bytes, f, sizeof f);
    } else {
        const sfac::PassDesc<float> f[2] = {fused_desc(p->r32[0], p->d32[0]), fused_desc(p->d32[dl], p->r32[dl])};
        memcpy(host.data() + p->off_desc, p->d32, sizeof(sfac::PassDesc<float>) * p->in.dims);
        memcpy(host.data() + p->off_desc + 3 * desc_bytes, p->r32, sizeof(sfac::PassDesc<float>) * p->in.dims);
        memcpy(host.data() + p->off_desc + 6 * desc_bytes, f, sizeof f);
    }
    e = hipMemcpy(p->dev, host.data(), p->dev_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p->dev);
        return hip_fail(e, "hipMemcpy tables");
    }
    if (p->in.lds_max > 64 * 1024) {
        e = dt == SFAC_FP64 ? sfac::allow_lds<double>(p->in.lds_max) : sfac::allow_lds<float>(p->in.lds_max);
        if (e != hipSuccess) {
            (void)hipFree(p->dev);
            return hip_fail(e, "hipFuncSetAttribute(max dynamic LDS)");
        }
    }
    *out = p.release();
    return SFAC_OK;
}

sfac_status sfac_step(sfac_plan p, void* u_dev, int64_t nsteps) {
    g_error.clear();
    if (!p) return fail(SFAC_EINVAL, "NULL plan");
    if (nsteps < 0) return fail(SFAC_EINVAL, "nsteps = %lld, expected >= 0", (long long)nsteps);
    if (!u_dev) return fail(SFAC_EINVAL, "NULL state pointer");
    const size_t es = p->in.dt == SFAC_FP64 ? 8 : 4;
    if (reinterpret_cast<uintptr_t>(u_dev) % es) return fail(SFAC_EINVAL, "state pointer not aligned to %zu bytes", es);
    if (nsteps == 0) return SFAC_OK;
    if (!p->use_graph) {
        p->set_u(u_dev);
        hipError_t e = p->launch_steps(p->stream, nsteps, p->parity);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        p->parity ^= (int)(nsteps & 1);
        return SFAC_OK;
    }
    if (p->graph_u != u_dev) {
        p->drop_graphs();
        p->set_u(u_dev);
        p->graph_u = u_dev;
    }
    // nsteps / chunk replays of the chunk-step graph, then one replay per set bit of the rest:
    // a call of fewer than chunk steps costs at most log2(chunk) + 1 graph launches
    const int64_t full = nsteps / p->chunk, rest = nsteps % p->chunk;
    hipGraphExec_t x = nullptr;
    // (an odd chunk alternates between the graphs of its two starting parities)
    for (int64_t k = 0; k < full; ++k) {
        const sfac_status st = p->graph_for(p->chunk, p->parity, &x);
        if (st != SFAC_OK) return st;
        hipError_t e = hipGraphLaunch(x, p->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        p->parity ^= p->chunk & 1;
    }
    for (int b = 62; b >= 0; --b) {
        const int64_t part = int64_t(1) << b;
        if (!(rest & part)) continue;
        const sfac_status st = p->graph_for(part, p->parity, &x);
        if (st != SFAC_OK) return st;
        hipError_t e = hipGraphLaunch(x, p->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        p->parity ^= (int)(part & 1);
    }
    return SFAC_OK;
}

sfac_status sfac_plan_time_passes(sfac_plan p, void* u_dev, int32_t reps, float* ms) {
    g_error.clear();
    if (!p) return fail(SFAC_EINVAL, "NULL plan");
    if (!u_dev || !ms || reps < 1) return fail(SFAC_EINVAL, "NULL state or output, or reps < 1");
    const size_t es = p->in.dt == SFAC_FP64 ? 8 : 4;
    if (reinterpret_cast<uintptr_t>(u_dev) % es) return fail(SFAC_EINVAL, "state pointer not aligned to %zu bytes", es);
    const int d = p->in.dims;
    const bool exact = p->exact != 0;
    // exact plans: an event pair around every dense product of `reps` whole steps; two-level
    // plans: one event pair around `reps` launches of one axis' pass replayed from a graph
    std::vector<hipEvent_t> ev(exact ? 2 * (size_t)d * reps : 2, nullptr);
    hipError_t e = hipSuccess;
    for (auto& x : ev) {
        e = hipEventCreate(&x);
        if (e != hipSuccess) break;
    }
    void* keep = p->graph_u;
    p->set_u(u_dev);
    if (exact) {
        for (int r = 0; r < reps && e == hipSuccess; ++r) {
            sfac::PassDesc<double> quiet = p->d64[d - 1];
            quiet.trace_part = nullptr;
            e = p->exact_step(p->stream, quiet, &ev[2 * (size_t)r * d]);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        for (int a = 0; a < d && e == hipSuccess; ++a) {
            double acc = 0;
            for (int r = 0; r < reps && e == hipSuccess; ++r) {
                const size_t i = 2 * ((size_t)r * d + a);
                float t = 0;
                e = hipEventElapsedTime(&t, ev[i], ev[i + 1]);
                acc += t;
            }
            ms[a] = (float)(acc / reps);
        }
    }
    if (!exact) e = hipStreamSynchronize(p->stream);
    if (!exact && e == hipSuccess) e = p->capture_stream();
    for (int a = 0; a < d && !exact && e == hipSuccess; ++a) {
        // plain launches outside sfac_step: not part of the per-step record
        sfac::PassDesc<double> d64 = p->d64[a];
        sfac::PassDesc<float> d32 = p->d32[a];
        d64.trace_part = nullptr;
        d32.trace_part = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        e = hipStreamBeginCapture(p->capture, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) break;
        hipError_t le = hipSuccess;
        for (int r = 0; r < reps && le == hipSuccess; ++r)
            le = p->in.dt == SFAC_FP64 ? launch_pass(d64, p->in.ax[a].lds, p->capture)
                                       : launch_pass(d32, p->in.ax[a].lds, p->capture);
        e = hipStreamEndCapture(p->capture, &graph);
        if (le != hipSuccess) e = le;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e == hipSuccess) e = sfac::launch_timing_mark(a + 1, p->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[0], p->stream);
        if (e == hipSuccess) e = hipGraphLaunch(exec, p->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[1], p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        float t = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, ev[0], ev[1]);
        if (e == hipSuccess) ms[a] = t / reps;
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
    if (!exact && e == hipSuccess) e = sfac::launch_timing_mark(0, p->stream);
    for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
    // the captured step graphs keep their own copies of the launch arguments
    if (keep) p->set_u(keep);
    return e == hipSuccess ? SFAC_OK : hip_fail(e, "timed pass launches");
}

sfac_status sfac_plan_time_fused(sfac_plan p, void* u_dev, int32_t reps, float* ms) {
    g_error.clear();
    if (!p) return fail(SFAC_EINVAL, "NULL plan");
    if (!u_dev || !ms || reps < 1) return fail(SFAC_EINVAL, "NULL state or output, or reps < 1");
    const size_t es = p->in.dt == SFAC_FP64 ? 8 : 4;
    if (reinterpret_cast<uintptr_t>(u_dev) % es) return fail(SFAC_EINVAL, "state pointer not aligned to %zu bytes", es);
    ms[0] = ms[1] = 0.0f;
    if (p->exact) return SFAC_OK;
    const int d = p->in.dims;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    void* keep = p->graph_u;
    p->set_u(u_dev);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e == hipSuccess) e = p->capture_stream();
    // [0]: axis 1, the last pass of a step in the order d..1 with the first of the next; [1]: axis d,
    // the last pass of a step in the order 1..d with the first of the next (as sfac_step fuses them)
    const int axes[2] = {0, d - 1};
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        const int a = axes[i];
        sfac::PassDesc<double> d64 = i == 0 ? fused_desc(p->r64[a], p->d64[a]) : fused_desc(p->d64[a], p->r64[a]);
        sfac::PassDesc<float> d32 = i == 0 ? fused_desc(p->r32[a], p->d32[a]) : fused_desc(p->d32[a], p->r32[a]);
        if (p->in.dt == SFAC_FP64 ? !can_fuse(d64) : !can_fuse(d32)) continue;
        d64.trace_part = nullptr;
        d32.trace_part = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        e = hipStreamBeginCapture(p->capture, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) break;
        hipError_t le = hipSuccess;
        for (int r = 0; r < reps && le == hipSuccess; ++r)
            le = p->in.dt == SFAC_FP64 ? launch_pass(d64, p->in.ax[a].lds, p->capture)
                                       : launch_pass(d32, p->in.ax[a].lds, p->capture);
        e = hipStreamEndCapture(p->capture, &graph);
        if (le != hipSuccess) e = le;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e == hipSuccess) e = sfac::launch_timing_mark(sfac::kFusedMark + a + 1, p->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[0], p->stream);
        if (e == hipSuccess) e = hipGraphLaunch(exec, p->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[1], p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        float t = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, ev[0], ev[1]);
        if (e == hipSuccess) ms[i] = t / reps;
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (d == 1) {
            ms[1] = ms[0];
            break;
        }
    }
    if (e == hipSuccess) e = sfac::launch_timing_mark(0, p->stream);
    for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
    if (keep) p->set_u(keep);
    return e == hipSuccess ? SFAC_OK : hip_fail(e, "timed fused launches");
}

sfac_status sfac_plan_destroy(sfac_plan p) {
    g_error.clear();
    if (!p) return SFAC_OK;
    (void)hipStreamSynchronize(p->stream);
    p->drop_graphs();
    if (p->capture) (void)hipStreamDestroy(p->capture);
    if (p->dev) (void)hipFree(p->dev);
    if (p->energy_dev) (void)hipFree(p->energy_dev);
    if (p->trace_dev) (void)hipFree(p->trace_dev);
    delete p;
    return SFAC_OK;
}


sfac_status sfac_plan_energy(sfac_plan p, const void* u_dev, double* energy) {
    g_error.clear();
    if (!p) return fail(SFAC_EINVAL, "NULL plan");
    if (!u_dev || !energy) return fail(SFAC_EINVAL, "NULL state or output");
    const size_t es = p->in.dt == SFAC_FP64 ? 8 : 4;
    if (reinterpret_cast<uintptr_t>(u_dev) % es) return fail(SFAC_EINVAL, "state pointer not aligned to %zu bytes", es);
    if (!p->energy_dev) {
        const sfac_status st = p->in.dt == SFAC_FP64 ? energy_setup<double>(p) : energy_setup<float>(p);
        if (st != SFAC_OK) return st;
    }
    // the kernels only read the state
    hipError_t e = p->in.dt == SFAC_FP64 ? energy_launch<double>(p, static_cast<double*>(const_cast<void*>(u_dev)))
                                         : energy_launch<float>(p, static_cast<float*>(const_cast<void*>(u_dev)));
    double sums[2] = {0.0, 0.0};
    if (e == hipSuccess) e = hipMemcpyAsync(sums, p->energy_dev, sizeof sums, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "energy");
    double hprod = 1.0;
    for (int a = 0; a < p->in.dims; ++a) hprod *= p->in.h[a];
    *energy = hprod * (sums[1] - 0.5 * sums[0]);
    return SFAC_OK;
}

sfac_status sfac_plan_trace(sfac_plan p, int64_t capacity) {
    g_error.clear();
    if (!p) return fail(SFAC_EINVAL, "NULL plan");
    if (capacity < 0 || capacity > (int64_t(1) << 40)) return fail(SFAC_EINVAL, "capacity = %lld", (long long)capacity);
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    p->drop_graphs();     // the step graphs gain or lose the step-index kernel
    if (p->trace_dev) (void)hipFree(p->trace_dev);
    p->trace_dev = nullptr;
    p->trace_cap = 0;
    p->trace_parts = 0;
    if (capacity > 0) {
        // one slot per wavefront of the launch that stores the statistics: the pass of axis d in
        // steps of the order 1..d, of axis 1 in steps of the order d..1
        auto slots = [p](int a, int* wpb) {
            long long blocks = p->in.dt == SFAC_FP64 ? sfac::pass_blocks(p->d64[a]) : sfac::pass_blocks(p->d32[a]);
            int threads = p->in.dt == SFAC_FP64 ? p->d64[a].threads : p->d32[a].threads;
            if (p->exact) {   // the closing nonlinear half-step kernel stores the statistics
                threads = sfac::kExactNlThreads;
                blocks = (p->in.points() + threads - 1) / threads;
            }
            *wpb = (threads + 63) / 64;
            return blocks * *wpb;
        };
        p->trace_parts = std::max(slots(p->in.dims - 1, &p->trace_wpb_last), slots(0, &p->trace_wpb_first));
        const size_t bytes = 8 + 8 * (size_t)capacity + 8 * (size_t)p->trace_parts;
        e = hipMalloc(&p->trace_dev, bytes);
        if (e != hipSuccess) {
            p->trace_dev = nullptr;
            p->set_trace();
            return e == hipErrorOutOfMemory ? fail(SFAC_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e))
                                            : hip_fail(e, "hipMalloc");
        }
        e = hipMemset(p->trace_dev, 0, bytes);
        if (e != hipSuccess) {
            (void)hipFree(p->trace_dev);
            p->trace_dev = nullptr;
            p->set_trace();
            return hip_fail(e, "hipMemset");
        }
        p->trace_cap = capacity;
    }
    p->set_trace();
    return SFAC_OK;
}

sfac_status sfac_plan_read_trace(sfac_plan p, double* out, int64_t capacity, int64_t* recorded) {
    g_error.clear();
    if (!p) return fail(SFAC_EINVAL, "NULL plan");
    if (!recorded || capacity < 0 || (capacity > 0 && !out)) return fail(SFAC_EINVAL, "NULL output or capacity < 0");
    *recorded = 0;
    if (!p->trace_dev) return SFAC_OK;
    hipError_t e = hipStreamSynchronize(p->stream);
    long long steps = 0;
    if (e == hipSuccess) e = hipMemcpy(&steps, p->trace_step(), sizeof steps, hipMemcpyDeviceToHost);
    const long long n = std::min<long long>(std::min<long long>(steps, p->trace_cap), capacity);
    if (e == hipSuccess && n > 0) {
        std::vector<unsigned long long> bits((size_t)n);
        e = hipMemcpy(bits.data(), p->trace_rec(), 8 * (size_t)n, hipMemcpyDeviceToHost);
        for (long long i = 0; e == hipSuccess && i < n; ++i) memcpy(&out[i], &bits[(size_t)i], 8);
    }
    if (e != hipSuccess) return hip_fail(e, "trace");
    *recorded = steps;
    return SFAC_OK;
}

size_t sfac_plan_device_bytes(sfac_plan p) { return p ? p->dev_bytes : 0; }

sfac_status sfac_plan_flags(sfac_plan p, uint32_t* flags, double* max_abs) {
    g_error.clear();
    if (!p) return fail(SFAC_EINVAL, "NULL plan");
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    unsigned char buf[16];
    e = hipMemcpy(buf, p->dev + p->off_stat, 16, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy status");
    unsigned long long bits;
    unsigned int fl;
    memcpy(&bits, buf, 8);
    memcpy(&fl, buf + 8, 4);
    if (flags) *flags = fl;
    if (max_abs) memcpy(max_abs, &bits, 8);
    return SFAC_OK;
}

sfac_status sfac_plan_reset_flags(sfac_plan p) {
    g_error.clear();
    if (!p) return fail(SFAC_EINVAL, "NULL plan");
    hipError_t e = sfac::launch_zero_words(reinterpret_cast<unsigned int*>(p->dev + p->off_stat), 4, p->stream);
    return e == hipSuccess ? SFAC_OK : hip_fail(e, "status clear");
}

sfac_status sfac_plan_method(sfac_plan p, int32_t axis, int32_t* method, int32_t* length) {
    g_error.clear();
    if (!p) return fail(SFAC_EINVAL, "NULL plan");
    if (axis < 1 || axis > p->in.dims) return fail(SFAC_EINVAL, "axis %d outside 1..%d", axis, p->in.dims);
    if (method) *method = p->exact ? SFAC_METHOD_EXACT : p->in.ax[axis - 1].host.method;
    if (length) *length = p->exact ? p->in.n[axis - 1] : p->in.ax[axis - 1].host.length;
    return SFAC_OK;
}

sfac_status sfac_axis_tables(int32_t n, double alpha, double eps, double tau, double h, int32_t method,
                             int32_t* length, double* scale_c, double* scale_s, int32_t* radices,
                             int32_t* nstages) {
    g_error.clear();
    int32_t ns[1] = {n};
    double al[1] = {alpha}, hs[1] = {h};
    sfac_status st = validate_instance(1, ns, al, eps, tau, hs, "");
    if (st != SFAC_OK) return st;
    const bool increment = (method & SFAC_TABLES_INCREMENT) != 0;
    int m = method & ~SFAC_TABLES_INCREMENT;
    if (m == SFAC_METHOD_AUTO) m = sfac::auto_method(n, SFAC_FP64);
    if (m != SFAC_METHOD_DIAG && m != SFAC_METHOD_EMBED) return fail(SFAC_EUNSUPPORTED, "no method for N = %d", n);
    sfac::AxisTables t;
    std::string err = sfac::build_axis_tables(sfac::AxisParams{n, alpha, eps, tau, h}, m, &t, 4, true, increment);
    if (!err.empty()) return fail(SFAC_EUNSUPPORTED, "%s", err.c_str());
    if (length) *length = t.length;
    if (scale_c) std::copy(t.scale_c.begin(), t.scale_c.end(), scale_c);
    if (scale_s) std::copy(t.scale_s.begin(), t.scale_s.end(), scale_s);
    if (radices) std::copy(t.radices.begin(), t.radices.end(), radices);
    if (nstages) *nstages = (int32_t)t.radices.size();
    return SFAC_OK;
}

sfac_status sfac_exact_exponential(int32_t n, double alpha, double eps, double tau, double h, double* P) {
    g_error.clear();
    if (!P) return fail(SFAC_EINVAL, "NULL output");
    int32_t ns[1] = {n};
    double al[1] = {alpha}, hs[1] = {h};
    sfac_status st = validate_instance(1, ns, al, eps, tau, hs, "");
    if (st != SFAC_OK) return st;
    std::vector<double> m;
    const std::string err = sfac::build_exact_exponential(sfac::AxisParams{n, alpha, eps, tau, h}, &m);
    if (!err.empty()) return fail(SFAC_EUNSUPPORTED, "%s", err.c_str());
    std::copy(m.begin(), m.end(), P);
    return SFAC_OK;
}

}  // extern "C"

// ===================================================================== groups
// A group steps any set of plans together: each plan makes the launches a lone sfac_step would
// make inside one step graph (its passes in its step orders, step boundaries fused where its
// kernel fuses), and the plans' i-th launches share one launch per (arithmetic, kernel variant)
// covering every plan that needs it. A launch's instances travel in its kernel
// arguments (sfac::GroupArgs: the device copy of each plan's pass descriptor and its state), so
// a group owns no device memory, a call never waits for the previous one, and a captured step
// graph stays valid for as long as its plans live. Step graphs are cached per set of (plan,
// state) pairs: a served tick with the same requests as the one before replays the same graph.
namespace {

struct GroupLaunch {
    int pass = 0, fp64 = 0, kind = 0, variant = 0, threads = 0;
    size_t lds = 0;
    sfac::GroupArgs<double> a64{};
    sfac::GroupArgs<float> a32{};
};

// One cached step graph: the (plan id, state) pairs of a phase, in call order.
struct GroupGraph {
    std::vector<std::pair<unsigned long long, void*>> key;
    int steps = 1;   // steps captured in the graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// A phase of at least kLongPhase steps replays a graph of kPhaseChunk steps first: fewer graph
// launches, and so fewer gaps between them, and more fused step boundaries on long batched runs;
// shorter phases (a served tick) and the remainder replay a graph of two steps, then one of one
// step if the count is odd.
constexpr int kPhaseChunk = 32;
constexpr int64_t kLongPhase = 64;

}  // namespace

struct sfac_group_s {
    static constexpr int kAux = 4;         // streams the launches of one pass fan out to
    static constexpr size_t kCache = 32;   // step graphs kept (most recently used first)
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;         // private streams used only while capturing a step
    hipStream_t aux[kAux] = {};
    hipEvent_t fork = nullptr, join[kAux] = {};
    std::list<GroupGraph> cache;

    static void destroy(GroupGraph& gg) {
        if (gg.exec) (void)hipGraphExecDestroy(gg.exec);
        if (gg.graph) (void)hipGraphDestroy(gg.graph);
        gg.exec = nullptr;
        gg.graph = nullptr;
    }
    hipError_t ensure_streams() {
        hipError_t e = hipSuccess;
        if (!capture) e = hipStreamCreateWithFlags(&capture, hipStreamNonBlocking);
        for (int k = 0; k < kAux && e == hipSuccess; ++k)
            if (!aux[k]) e = hipStreamCreateWithFlags(&aux[k], hipStreamNonBlocking);
        if (e == hipSuccess && !fork) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        for (int k = 0; k < kAux && e == hipSuccess; ++k)
            if (!join[k]) e = hipEventCreateWithFlags(&join[k], hipEventDisableTiming);
        return e;
    }
    void release() {
        for (auto& gg : cache) destroy(gg);
        cache.clear();
        if (fork) (void)hipEventDestroy(fork);
        for (int k = 0; k < kAux; ++k) {
            if (join[k]) (void)hipEventDestroy(join[k]);
            if (aux[k]) (void)hipStreamDestroy(aux[k]);
        }
        if (capture) (void)hipStreamDestroy(capture);
    }
};

namespace {

// The plans of a phase that step (in call order), with their states and the parity of the
// steps each plan had queued when the phase began (its first step's axis order).
struct PhaseEntry {
    sfac_plan plan;
    void* u;
    int parity;
};

template <typename T>
const sfac::PassDesc<T>& host_desc(const sfac_plan_s* p, int a) {
    if constexpr (std::is_same<T, double>::value)
        return p->d64[a];
    else
        return p->d32[a];
}
template <typename T>
sfac::GroupArgs<T>& launch_args(GroupLaunch& l) {
    if constexpr (std::is_same<T, double>::value)
        return l.a64;
    else
        return l.a32;
}

// One launch of one plan in a grouped graph: the pass over `axis` (`which` 0: the descriptor for
// steps in the order 1..d, 1: in the order d..1) or, `which` 2 and 3, the two passes over axis 1
// (after a step in the order d..1) or axis d (after one in the order 1..d) in one launch.
struct PlanLaunch {
    const PhaseEntry* e;
    int axis;
    int which;
};

// The launches each plan of a phase makes in `steps` steps, as a lone sfac_step makes them inside
// one graph: its passes in its step orders, a step boundary inside the graph fused where the
// plan's kernel fuses. out[i] holds every plan's i-th launch; plans are independent, so the
// launches of one index may run in any order among themselves.
void phase_slots(const std::vector<PhaseEntry>& entries, int steps, std::vector<std::vector<PlanLaunch>>* out) {
    out->clear();
    for (const PhaseEntry& e : entries) {
        const sfac_plan p = e.plan;
        const int dims = p->in.dims;
        size_t idx = 0;
        bool carried = false;
        auto push = [&](PlanLaunch l) {
            if (out->size() <= idx) out->resize(idx + 1);
            (*out)[idx++].push_back(l);
        };
        for (int j = 0; j < steps; ++j) {
            const int odd = (e.parity + j) & 1;
            for (int pos = 0; pos < dims; ++pos) {
                const int a = odd ? dims - 1 - pos : pos;
                if (pos == 0 && carried) {
                    carried = false;
                    continue;
                }
                const bool fusable = p->in.dt == SFAC_FP64 ? can_fuse(p->d64[a]) : can_fuse(p->d32[a]);
                if (pos == dims - 1 && j + 1 < steps && fusable) {
                    push(PlanLaunch{&e, a, odd ? 2 : 3});
                    carried = true;
                } else {
                    push(PlanLaunch{&e, a, odd});
                }
            }
        }
    }
}

// The grouped launches of one slot for the plans of arithmetic T: one launch per kernel variant
// (single or two-pass), at most kGroupSlots instances each.
template <typename T>
void slot_launches(const std::vector<PlanLaunch>& slot, int index, std::vector<GroupLaunch>* out) {
    constexpr bool f64 = std::is_same<T, double>::value;
    std::vector<std::pair<int, int>> keys;   // (kernel kind, variant): see launch_axis_pass_multi
    std::vector<std::vector<const PlanLaunch*>> members;
    for (const PlanLaunch& pl : slot) {
        sfac_plan p = pl.e->plan;
        if ((p->in.dt == SFAC_FP64) != f64) continue;
        const sfac::PassDesc<T>& d = host_desc<T>(p, pl.axis);
        const int kind = d.method == SFAC_METHOD_EMBED ? 1 : (d.d2a > 0 ? 2 : 0);
        const int variant = (kind == 1 ? d.log2m * 8 + d.log2e + (d.stage ? 128 : 0)
                                       : (kind == 2 ? d.d2a * 64 + d.d2b + (d.d2wave ? 4096 : 0) : 0)) +
                            (pl.which >= 2 ? sfac::kTwiceVariant : 0);
        const std::pair<int, int> key(kind, variant);
        const size_t g = std::find(keys.begin(), keys.end(), key) - keys.begin();
        if (g == keys.size()) {
            keys.push_back(key);
            members.emplace_back();
        }
        members[g].push_back(&pl);
    }
    for (size_t g = 0; g < keys.size(); ++g) {
        for (size_t first = 0; first < members[g].size(); first += sfac::kGroupSlots) {
            const size_t last = std::min(members[g].size(), first + sfac::kGroupSlots);
            GroupLaunch l;
            l.pass = index;
            l.fp64 = f64;
            l.kind = keys[g].first;
            l.variant = keys[g].second;
            sfac::GroupArgs<T>& args = launch_args<T>(l);
            args.n = (int)(last - first);
            args.start[0] = 0;
            size_t lds = 0;
            int threads = l.kind == 0 ? sfac::kBlockThreads : 0;
            for (size_t i = first; i < last; ++i) {
                const PlanLaunch& pl = *members[g][i];
                sfac_plan p = pl.e->plan;
                const sfac::PassDesc<T>& d = host_desc<T>(p, pl.axis);
                const int k = (int)(i - first);
                args.desc[k] = pl.which >= 2 ? p->template fused_device_desc<T>(pl.which - 2)
                                             : p->template device_desc<T>(pl.axis, pl.which);
                args.u[k] = static_cast<T*>(pl.e->u);
                args.start[k + 1] = args.start[k] + sfac::pass_blocks(d);
                lds = std::max(lds, p->in.ax[pl.axis].lds);
                if (l.kind != 0) threads = std::max(threads, d.threads);
            }
            const int v = l.variant % sfac::kTwiceVariant;
            if (l.kind == 1) {
                const int E = 1 << sfac::embed_log2e((v % 128) / 8, v % 8);
                lds = (size_t)threads * E * sizeof(sfac::cplx<T>);
            } else if (l.kind == 2) {
                // a full block of P-thread lines (or of wavefronts of 64/P lines); lines beyond
                // a descriptor's lpb idle
                const int A = (v % 4096) / 64, B = v % 64, P = std::max(A, B);
                const int lines = v >= 4096 ? (threads / 64) * (64 / P) : threads / P;
                lds = (size_t)lines * sfac::diag2_line_stride(A, B, sizeof(sfac::cplx<T>)) * sizeof(sfac::cplx<T>);
            }
            l.threads = threads;
            l.lds = lds;
            out->push_back(l);
        }
    }
}

hipError_t group_launch(const GroupLaunch& l, hipStream_t s) {
    return l.fp64 ? sfac::launch_axis_pass_multi<double>(l.kind, l.variant, l.threads, l.a64, l.lds, s)
                  : sfac::launch_axis_pass_multi<float>(l.kind, l.variant, l.threads, l.a32, l.lds, s);
}

// Captures the launches of a phase's graph slot after slot; the launches of one slot (different
// kernel variants and arithmetic, disjoint plans) fan out over the auxiliary streams and join
// before the next slot, so every plan still sees its launches in order.
sfac_status capture_step(sfac_group g, const std::vector<GroupLaunch>& launches, int slots, hipGraph_t* graph) {
    *graph = nullptr;
    hipError_t e = hipStreamBeginCapture(g->capture, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = hipSuccess;
    for (int slot = 0; slot < slots && le == hipSuccess; ++slot) {
        std::vector<const GroupLaunch*> ls;
        for (const GroupLaunch& l : launches)
            if (l.pass == slot) ls.push_back(&l);
        if (ls.empty()) continue;
        if (ls.size() == 1) {
            le = group_launch(*ls[0], g->capture);
            continue;
        }
        le = hipEventRecord(g->fork, g->capture);
        const int used = (int)std::min<size_t>(ls.size(), sfac_group_s::kAux);
        for (int k = 0; k < used && le == hipSuccess; ++k) le = hipStreamWaitEvent(g->aux[k], g->fork, 0);
        for (size_t k = 0; k < ls.size() && le == hipSuccess; ++k) le = group_launch(*ls[k], g->aux[k % sfac_group_s::kAux]);
        for (int k = 0; k < used && le == hipSuccess; ++k) le = hipEventRecord(g->join[k], g->aux[k]);
        for (int k = 0; k < used && le == hipSuccess; ++k) le = hipStreamWaitEvent(g->capture, g->join[k], 0);
    }
    e = hipStreamEndCapture(g->capture, graph);
    if (le != hipSuccess || e != hipSuccess) {
        if (e == hipSuccess && *graph) (void)hipGraphDestroy(*graph);
        *graph = nullptr;
        return le != hipSuccess ? hip_fail(le, "grouped kernel launch during capture")
                                : hip_fail(e, "hipStreamEndCapture");
    }
    return SFAC_OK;
}

// The step graph of a phase: from the cache, or captured and instantiated (the least recently
// used graph is dropped once the cache is full, after the stream has finished with it).
sfac_status phase_graph(sfac_group g, const std::vector<PhaseEntry>& entries, int steps, hipGraphExec_t* exec) {
    std::vector<std::pair<unsigned long long, void*>> key;
    key.reserve(entries.size());
    for (const PhaseEntry& e : entries) key.emplace_back(2 * e.plan->id + (unsigned long long)e.parity, e.u);
    for (auto it = g->cache.begin(); it != g->cache.end(); ++it)
        if (it->key == key && it->steps == steps) {
            g->cache.splice(g->cache.begin(), g->cache, it);
            *exec = g->cache.front().exec;
            return SFAC_OK;
        }
    std::vector<std::vector<PlanLaunch>> slots;
    phase_slots(entries, steps, &slots);
    std::vector<GroupLaunch> launches;
    for (size_t i = 0; i < slots.size(); ++i) {
        slot_launches<double>(slots[i], (int)i, &launches);
        slot_launches<float>(slots[i], (int)i, &launches);
    }
    size_t lds_need = 0;
    for (const auto& l : launches) lds_need = std::max(lds_need, l.lds);
    if (lds_need > 64 * 1024) {
        hipError_t e = sfac::allow_lds<double>(lds_need);
        if (e == hipSuccess) e = sfac::allow_lds<float>(lds_need);
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(max dynamic LDS)");
    }
    hipError_t e = g->ensure_streams();
    if (e != hipSuccess) return hip_fail(e, "group streams and events");
    GroupGraph gg;
    gg.key = std::move(key);
    gg.steps = steps;
    sfac_status st = capture_step(g, launches, (int)slots.size(), &gg.graph);
    if (st != SFAC_OK) return st;
    e = hipGraphInstantiate(&gg.exec, gg.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        sfac_group_s::destroy(gg);
        return hip_fail(e, "hipGraphInstantiate");
    }
    if (g->cache.size() >= sfac_group_s::kCache) {
        e = hipStreamSynchronize(g->stream);   // the dropped graph may still be running
        if (e != hipSuccess) {
            sfac_group_s::destroy(gg);
            return hip_fail(e, "hipStreamSynchronize");
        }
        sfac_group_s::destroy(g->cache.back());
        g->cache.pop_back();
    }
    g->cache.push_front(std::move(gg));
    *exec = g->cache.front().exec;
    return SFAC_OK;
}

sfac_status group_run(sfac_group g, int32_t count, const sfac_plan* plans, void* const* u_dev,
                      const int64_t* nsteps) {
    std::vector<PhaseEntry> all;
    std::vector<int64_t> steps, bounds;
    for (int32_t i = 0; i < count; ++i) {
        sfac_plan p = plans[i];
        if (!p) return fail(SFAC_EINVAL, "plan %d is NULL", i);
        if (p->exact) return fail(SFAC_EUNSUPPORTED, "plan %d: a plan of the exact exponential steps alone", i);
        if (nsteps[i] < 0) return fail(SFAC_EINVAL, "plan %d: nsteps = %lld", i, (long long)nsteps[i]);
        if (nsteps[i] == 0) continue;
        const size_t es = p->in.dt == SFAC_FP64 ? 8 : 4;
        if (!u_dev[i]) return fail(SFAC_EINVAL, "plan %d: NULL state pointer", i);
        if (reinterpret_cast<uintptr_t>(u_dev[i]) % es) return fail(SFAC_EINVAL, "plan %d: misaligned state", i);
        for (int32_t j = 0; j < i; ++j)
            if (plans[j] == p && nsteps[j] > 0) return fail(SFAC_EINVAL, "plan %d appears twice", i);
        all.push_back(PhaseEntry{p, u_dev[i], 0});
        steps.push_back(nsteps[i]);
        bounds.push_back(nsteps[i]);
    }
    if (bounds.empty()) return SFAC_OK;
    std::sort(bounds.begin(), bounds.end());
    bounds.erase(std::unique(bounds.begin(), bounds.end()), bounds.end());
    // phase after phase (the maximal step ranges with a fixed set of active plans): graphs of
    // kPhaseChunk steps on long phases, then of two steps, then of one (an even number of steps
    // leaves every plan's axis order where it was)
    int64_t done = 0;
    for (const int64_t bound : bounds) {
        std::vector<PhaseEntry> active;
        for (size_t i = 0; i < all.size(); ++i)
            if (steps[i] >= bound) {
                active.push_back(all[i]);
                active.back().parity = all[i].plan->parity;
            }
        int64_t left = bound - done;
        auto replay = [&](int graph_steps, int64_t times) -> sfac_status {
            if (times <= 0) return SFAC_OK;
            hipGraphExec_t exec = nullptr;
            const sfac_status st = phase_graph(g, active, graph_steps, &exec);
            if (st != SFAC_OK) return st;
            for (int64_t r = 0; r < times; ++r) {
                const hipError_t e = hipGraphLaunch(exec, g->stream);
                if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
            }
            return SFAC_OK;
        };
        sfac_status st = SFAC_OK;
        if (left >= kLongPhase) {
            st = replay(kPhaseChunk, left / kPhaseChunk);
            left %= kPhaseChunk;
        }
        if (st == SFAC_OK) st = replay(2, left / 2);
        if (st == SFAC_OK) st = replay(1, left % 2);
        if (st != SFAC_OK) return st;
        for (PhaseEntry& e : active) e.plan->parity ^= (int)((bound - done) & 1);
        done = bound;
    }
    return SFAC_OK;
}

}  // namespace

// ===================================================================== batches
struct sfac_batch_s {
    std::vector<sfac_plan> plans;
    sfac_group group = nullptr;
};

extern "C" {

sfac_status sfac_group_create(sfac_group* out, void* hip_stream) {
    g_error.clear();
    if (!out) return fail(SFAC_EINVAL, "NULL output handle");
    *out = nullptr;
    sfac_group g = new (std::nothrow) sfac_group_s();
    if (!g) return fail(SFAC_ENOMEM, "host allocation failed");
    g->stream = static_cast<hipStream_t>(hip_stream);
    *out = g;
    return SFAC_OK;
}

sfac_status sfac_group_step(sfac_group g, int32_t count, const sfac_plan* plans, void* const* u_dev,
                            const int64_t* nsteps) {
    g_error.clear();
    if (!g) return fail(SFAC_EINVAL, "NULL group");
    if (count < 0 || (count > 0 && (!plans || !u_dev || !nsteps)))
        return fail(SFAC_EINVAL, "count = %d with NULL arrays", count);
    return group_run(g, count, plans, u_dev, nsteps);
}

sfac_status sfac_group_destroy(sfac_group g) {
    g_error.clear();
    if (!g) return SFAC_OK;
    (void)hipStreamSynchronize(g->stream);
    g->release();
    delete g;
    return SFAC_OK;
}

size_t sfac_group_device_bytes(sfac_group) { return 0; }

sfac_status sfac_batch_create(sfac_batch* out, int32_t count, const sfac_instance_desc* desc, sfac_dtype dt,
                              void* hip_stream, const sfac_options* opts) {
    g_error.clear();
    if (!out) return fail(SFAC_EINVAL, "NULL output handle");
    *out = nullptr;
    if (count < 1 || !desc) return fail(SFAC_EINVAL, "count = %d with %s descriptors", count, desc ? "" : "NULL");
    if (dt != SFAC_FP64 && dt != SFAC_FP32) return fail(SFAC_EINVAL, "unknown dtype %d", (int)dt);
    std::unique_ptr<sfac_batch_s> b(new (std::nothrow) sfac_batch_s());
    if (!b) return fail(SFAC_ENOMEM, "host allocation failed");
    for (int32_t i = 0; i < count; ++i) {
        const sfac_instance_desc& d = desc[i];
        sfac_options opt{};
        if (opts) opt = opts[i];
        opt.use_graph = 0;   // a batch steps through its group, never through a plan's graphs
        for (int a = 0; a < 3; ++a)
            if (opt.method[a] == SFAC_METHOD_EXACT) {
                for (sfac_plan q : b->plans) sfac_plan_destroy(q);
                return fail(SFAC_EUNSUPPORTED, "instance %d: the exact exponential is available to single plans only",
                            i);
            }
        sfac_plan p = nullptr;
        sfac_status st = sfac_plan_create(&p, d.dims, d.n, d.alpha, d.eps, d.tau, d.h, dt, hip_stream, &opt);
        if (st != SFAC_OK) {
            std::string msg = g_error;
            for (sfac_plan q : b->plans) sfac_plan_destroy(q);
            return fail(st, "instance %d: %s", i, msg.c_str());
        }
        b->plans.push_back(p);
    }
    sfac_status st = sfac_group_create(&b->group, hip_stream);
    if (st != SFAC_OK) {
        for (sfac_plan q : b->plans) sfac_plan_destroy(q);
        return st;
    }
    *out = b.release();
    return SFAC_OK;
}

sfac_status sfac_batch_step(sfac_batch b, void* const* u_dev, const int64_t* nsteps) {
    g_error.clear();
    if (!b) return fail(SFAC_EINVAL, "NULL batch");
    if (!u_dev || !nsteps) return fail(SFAC_EINVAL, "NULL state or step array");
    return group_run(b->group, (int32_t)b->plans.size(), b->plans.data(), u_dev, nsteps);
}

sfac_plan sfac_batch_plan(sfac_batch b, int32_t i) {
    if (!b || i < 0 || i >= (int32_t)b->plans.size()) return nullptr;
    return b->plans[i];
}

sfac_status sfac_batch_destroy(sfac_batch b) {
    g_error.clear();
    if (!b) return SFAC_OK;
    sfac_group_destroy(b->group);
    for (sfac_plan p : b->plans) sfac_plan_destroy(p);
    delete b;
    return SFAC_OK;
}

size_t sfac_batch_device_bytes(sfac_batch b) {
    if (!b) return 0;
    size_t s = sfac_group_device_bytes(b->group);
    for (sfac_plan p : b->plans) s += sfac_plan_device_bytes(p);
    return s;
}

}  // extern "C"

// ===================================================================== solve without allocation
// sfac_solve_noalloc keeps an instance's tables and its status words in `scratch`, a fixed
// array in device memory that the library image brings along (one copy per device, held until
// the process ends), so the call allocates nothing on the device. Host code reaches it only
// through the address hipGetSymbolAddress returns on each device: the array's name is a host
// stand-in, not a device address.
namespace {
constexpr size_t kScratchBytes = size_t(512) << 10;
constexpr int kScratchDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_lock;
void* g_scratch_ptr[kScratchDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
sfac_status scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kScratchDevices) return fail(SFAC_EUNSUPPORTED, "device %d: too many devices", dev);
    std::lock_guard<std::mutex> guard(g_scratch_lock);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(SFAC_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SFAC_OK;
}

template <typename T>
sfac_status noalloc_run(const Instance& in, unsigned char* base, size_t off_stat, T* u, int64_t nsteps,
                        hipStream_t s) {
    sfac::PassDesc<T> d[3], r[3];
    auto* smax = reinterpret_cast<unsigned long long*>(base + off_stat);
    auto* sflags = reinterpret_cast<unsigned int*>(base + off_stat + 8);
    for (int a = 0; a < in.dims; ++a) {
        d[a] = make_desc<T>(in, a, base, u, smax, sflags);
        r[a] = reversed_desc(d[a], a, in.dims);
    }
    // the kernels and axis orders of a new plan's sfac_step
    const hipError_t e = launch_sequence(d, r, in, 0, nsteps, true, s, [](hipStream_t) { return hipSuccess; });
    return e == hipSuccess ? SFAC_OK : hip_fail(e, "kernel launch");
}
}  // namespace

extern "C" sfac_status sfac_solve_noalloc(int32_t dims, const int32_t* n_axis, const double* alpha_axis, double eps,
                                          double tau, const double* h_axis, sfac_dtype dt, void* u_dev, int64_t nsteps,
                                          void* hip_stream, const sfac_options* opt, uint32_t* flags,
                                          double* max_abs) {
    g_error.clear();
    if (dt != SFAC_FP64 && dt != SFAC_FP32) return fail(SFAC_EINVAL, "unknown dtype %d", (int)dt);
    if (nsteps < 0) return fail(SFAC_EINVAL, "nsteps = %lld, expected >= 0", (long long)nsteps);
    if (!u_dev) return fail(SFAC_EINVAL, "NULL state pointer");
    const size_t es = dt == SFAC_FP64 ? 8 : 4;
    if (reinterpret_cast<uintptr_t>(u_dev) % es) return fail(SFAC_EINVAL, "state pointer not aligned to %zu bytes", es);
    if (opt) {
        for (int a = 0; a < 3; ++a) {
            if (opt->method[a] == SFAC_METHOD_EXACT)
                return fail(SFAC_EUNSUPPORTED, "the exact exponential needs a plan (its scratch state is allocated)");
            if (opt->method[a] < SFAC_METHOD_AUTO || opt->method[a] > SFAC_METHOD_EXACT)
                return fail(SFAC_EINVAL, "unknown method %d for axis %d", opt->method[a], a + 1);
            if (opt->lines_per_block[a] < 0 || opt->lines_per_block[a] > 256)
                return fail(SFAC_EINVAL, "lines_per_block = %d for axis %d, expected 0..256", opt->lines_per_block[a],
                            a + 1);
        }
    }
    Instance in;
    sfac_status st = build_instance(&in, dims, n_axis, alpha_axis, eps, tau, h_axis, dt, opt, "");
    if (st != SFAC_OK) return st;
    const size_t off_stat = align_up(in.table_bytes, 256);
    const size_t total = off_stat + 256;
    if (total > kScratchBytes)
        return fail(SFAC_EUNSUPPORTED, "the tables need %zu bytes, more than the %zu bytes of the static workspace",
                    total, kScratchBytes);
    void* base = nullptr;
    st = scratch_address(&base);
    if (st != SFAC_OK) return st;
    // tables and zeroed status words in one copy from host memory, ordered on the stream after
    // the work already queued there (an earlier call's passes read the same workspace)
    std::vector<unsigned char> host(total, 0);
    for (int a = 0; a < in.dims; ++a) {
        if (dt == SFAC_FP64)
            axis_table_fill<double>(in.ax[a].host, in.ax[a], host.data());
        else
            axis_table_fill<float>(in.ax[a].host, in.ax[a], host.data());
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipMemcpyAsync(base, host.data(), total, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync tables");
    if (in.lds_max > 64 * 1024) {
        e = dt == SFAC_FP64 ? sfac::allow_lds<double>(in.lds_max) : sfac::allow_lds<float>(in.lds_max);
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(max dynamic LDS)");
    }
    unsigned char* b = static_cast<unsigned char*>(base);
    st = dt == SFAC_FP64 ? noalloc_run<double>(in, b, off_stat, static_cast<double*>(u_dev), nsteps, s)
                         : noalloc_run<float>(in, b, off_stat, static_cast<float*>(u_dev), nsteps, s);
    if (st != SFAC_OK) return st;
    if (flags || max_abs) {
        unsigned char buf[16];
        e = hipMemcpyAsync(buf, b + off_stat, 16, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "status read-back");
        unsigned long long bits;
        unsigned int fl;
        memcpy(&bits, buf, 8);
        memcpy(&fl, buf + 8, 4);
        if (flags) *flags = fl;
        if (max_abs) memcpy(max_abs, &bits, 8);
    }
    return SFAC_OK;
}
