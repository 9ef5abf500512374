// Host stand-in for the HIP runtime, for a CPU build of the library's host code under
// AddressSanitizer and UndefinedBehaviorSanitizer: "device" memory is host memory, and every
// allocation, stream, event, stream capture and graph is tracked. Misuse aborts the process with a
// message: freeing what is not allocated, copies outside allocations, using destroyed streams,
// events, graphs or graph executables, waiting on an event of a finished capture, capturing on
// the legacy stream, copies or memsets recorded into a capture. Launches are validated when they
// run: at once, or for a captured launch at every replay of its graph (mock_kernels.cpp).
// With MOCK_FAIL_EVERY=k in the environment every k-th call of the fallible APIs (allocation,
// stream and event creation, copies, capture, instantiation, graph and kernel launches, stream
// synchronisation) fails the way the runtime reports it, so that the library's error paths run
// under the sanitizers too (a launch that fails inside a capture invalidates the capture).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <vector>
#include <functional>

struct MockGraph;
struct MockStream { MockGraph* cap = nullptr; bool alive = true; };
struct MockEvent { MockGraph* cap = nullptr; bool alive = true; };
struct MockGraph { std::vector<std::function<void()>> launches; std::set<MockStream*> joined; bool alive = true; bool invalid = false; };
struct MockExec { std::vector<std::function<void()>> launches; bool alive = true; };

static std::map<uintptr_t, size_t> g_alloc;   // device allocations (host memory here)
static std::set<void*> g_streams, g_events, g_graphs, g_execs;
[[noreturn]] void mock_die(const char* what) { fprintf(stderr, "MOCK HIP ERROR: %s\n", what); fflush(stderr); abort(); }

bool mock_range_live(const void* p, size_t n) {
    uintptr_t a = reinterpret_cast<uintptr_t>(p);
    auto it = g_alloc.upper_bound(a);
    if (it == g_alloc.begin()) return false;
    --it;
    return a >= it->first && a + n <= it->first + it->second;
}
static bool is_device(const void* p) {
    uintptr_t a = reinterpret_cast<uintptr_t>(p);
    auto it = g_alloc.upper_bound(a);
    if (it == g_alloc.begin()) return false;
    --it;
    return a < it->first + it->second;
}
static long g_fail_every = -1, g_fallible = 0, g_injected = 0;
// true when this fallible call is to fail
bool mock_inject() {
    if (g_fail_every < 0) {
        const char* e = getenv("MOCK_FAIL_EVERY");
        g_fail_every = e ? atol(e) : 0;
    }
    if (g_fail_every <= 0) return false;
    if (++g_fallible % g_fail_every) return false;
    ++g_injected;
    return true;
}
extern "C" size_t mock_injected_failures() { return (size_t)g_injected; }
extern "C" size_t mock_live_allocations() { return g_alloc.size(); }
extern "C" size_t mock_live_streams() { return g_streams.size(); }
extern "C" size_t mock_live_graphs() { return g_graphs.size() + g_execs.size(); }

static MockStream* check_stream(hipStream_t s) {
    if (s && !g_streams.count(s)) mock_die("use of a stream that does not exist");
    return s;
}
// a launch on stream s: recorded into the capture, or run (validated) at once
void mock_submit(hipStream_t s, std::function<void()> f) {
    check_stream(s);
    if (s && s->cap) s->cap->launches.push_back(std::move(f));
    else f();
}
// a launch that fails: inside a capture it invalidates the capture
hipError_t mock_fail_launch(hipStream_t s) {
    check_stream(s);
    if (s && s->cap) s->cap->invalid = true;
    return hipErrorInvalidValue;
}

hipError_t hipMalloc(void** p, size_t n) {
    if (mock_inject()) return hipErrorOutOfMemory;
    void* q = aligned_alloc(256, (n + 255) / 256 * 256);
    if (!q) return hipErrorOutOfMemory;
    if (n <= (1u << 20)) memset(q, 0xA5, (n + 255) / 256 * 256);
    g_alloc[reinterpret_cast<uintptr_t>(q)] = n;
    *p = q;
    return hipSuccess;
}
hipError_t hipFree(void* p) {
    if (!p) return hipSuccess;
    auto it = g_alloc.find(reinterpret_cast<uintptr_t>(p));
    if (it == g_alloc.end()) mock_die("hipFree of memory that is not a live allocation");
    g_alloc.erase(it);
    free(p);
    return hipSuccess;
}
static void check_copy(void* d, const void* s, size_t n, hipMemcpyKind k) {
    if ((k == hipMemcpyHostToDevice || k == hipMemcpyDeviceToDevice) && !mock_range_live(d, n)) mock_die("copy to a device range that is not allocated");
    if ((k == hipMemcpyDeviceToHost || k == hipMemcpyDeviceToDevice) && !mock_range_live(s, n)) mock_die("copy from a device range that is not allocated");
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k) {
    check_copy(d, s, n, k);
    if (mock_inject()) return hipErrorInvalidValue;
    memcpy(d, s, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st) {
    check_copy(d, s, n, k);
    if (st && st->cap) mock_die("copy recorded into a capture");
    if (mock_inject()) return hipErrorInvalidValue;
    memcpy(d, s, n);
    return hipSuccess;
}
hipError_t hipMemset(void* d, int v, size_t n) { if (!mock_range_live(d, n)) mock_die("memset out of range"); memset(d, v, n); return hipSuccess; }
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st) {
    if (st && st->cap) mock_die("memset recorded into a capture");
    return hipMemset(d, v, n);
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    if (mock_inject()) return hipErrorOutOfMemory;
    *s = new MockStream();
    g_streams.insert(*s);
    return hipSuccess;
}
hipError_t hipStreamCreate(hipStream_t* s) { return hipStreamCreateWithFlags(s, 0); }
hipError_t hipStreamDestroy(hipStream_t s) {
    if (!g_streams.count(s)) mock_die("hipStreamDestroy of a stream that does not exist");
    if (s->cap) mock_die("hipStreamDestroy of a stream in capture");
    g_streams.erase(s);
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    check_stream(s);
    if (s && s->cap) mock_die("synchronize of a capturing stream");
    if (mock_inject()) return hipErrorIllegalState;
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
    if (mock_inject()) return hipErrorOutOfMemory;
    *e = new MockEvent();
    g_events.insert(*e);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    if (!g_events.count(e)) mock_die("hipEventDestroy of an event that does not exist");
    g_events.erase(e);
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    if (!g_events.count(e)) mock_die("record of an event that does not exist");
    check_stream(s);
    e->cap = s ? s->cap : nullptr;
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    if (!g_events.count(a) || !g_events.count(b)) mock_die("elapsed time of events that do not exist");
    *ms = 0.01f;
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
    check_stream(s);
    if (!g_events.count(e)) mock_die("wait on an event that does not exist");
    if (e->cap) {
        if (!g_graphs.count(e->cap)) mock_die("wait on an event recorded in a finished capture");
        if (s && !s->cap) { s->cap = e->cap; e->cap->joined.insert(s); }
    }
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    if (!s) mock_die("capture on the legacy default stream");
    check_stream(s);
    if (s->cap) mock_die("begin capture on a stream already capturing");
    if (mock_inject()) return hipErrorStreamCaptureUnsupported;
    s->cap = new MockGraph();
    g_graphs.insert(s->cap);
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
    check_stream(s);
    if (!s->cap) mock_die("end capture on a stream not capturing");
    MockGraph* gr = s->cap;
    s->cap = nullptr;
    // a joined stream is back when its last record was joined into the origin (the mock only
    // requires that no joined stream still has launches queued after its join: checked loosely)
    for (MockStream* j : gr->joined) j->cap = nullptr;
    gr->joined.clear();
    if (gr->invalid || mock_inject()) {   // the capture ends either way; no graph is returned
        g_graphs.erase(gr);
        delete gr;
        *g = nullptr;
        return hipErrorStreamCaptureInvalidated;
    }
    *g = gr;
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
    if (!g_graphs.count(g)) mock_die("instantiate of a graph that does not exist");
    if (mock_inject()) return hipErrorOutOfMemory;
    *x = new MockExec();
    (*x)->launches = g->launches;
    g_execs.insert(*x);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
    if (!g_execs.count(x)) mock_die("launch of a graph exec that does not exist");
    check_stream(s);
    if (s && s->cap) mock_die("graph launch into a capture");
    if (mock_inject()) return hipErrorInvalidValue;
    for (auto& f : x->launches) f();
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
    if (!g_execs.count(x)) mock_die("destroy of a graph exec that does not exist");
    g_execs.erase(x);
    delete x;
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    if (!g_graphs.count(g)) mock_die("destroy of a graph that does not exist");
    g_graphs.erase(g);
    delete g;
    return hipSuccess;
}
const char* hipGetErrorString(hipError_t) { return "mock error"; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = const_cast<void*>(sym); return hipSuccess; }
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }

extern "C" void* mock_alloc(size_t n) { void* p = nullptr; return hipMalloc(&p, n) == hipSuccess ? p : nullptr; }
extern "C" void mock_free(void* p) { hipFree(p); }
