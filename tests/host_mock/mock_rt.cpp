// A validating CPU stand-in for the HIP and rocFFT calls the library's host
// code makes.  "Device" memory is host memory; kernels are stubs that only
// record a node on their stream.  Every stream, event, graph and FFT handle is
// checked for validity, and stream capture is modelled as a dependency graph:
// a capturing stream may not synchronise or wait on an event recorded outside
// the capture, and at the end of a capture every stream forked into it must
// have joined back into the origin stream.  Any violation prints a backtrace
// and aborts.  Built with AddressSanitizer, this checks the host logic of the
// library (workspace carving, batch scheduling, graph capture) on a CPU.
#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <execinfo.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <vector>

#define FAIL(...)                                                  \
    do {                                                           \
        std::fprintf(stderr, "MOCK ERROR: " __VA_ARGS__);          \
        std::fprintf(stderr, "\n");                                \
        void* bt_[40];                                             \
        backtrace_symbols_fd(bt_, backtrace(bt_, 40), 2);          \
        std::abort();                                              \
    } while (0)

struct Capture {
    MockStream* origin;
    std::vector<std::vector<int>> deps;   // node -> the nodes it depends on
    bool open;
};
struct MockStream {
    int capture = 0;                      // capture id, 0 when not capturing
    std::vector<int> frontier;            // last captured nodes of this stream
};
struct MockEvent {
    bool recorded = false;
    int capture = 0;
    std::vector<int> nodes;
    unsigned flags = 0;
};
struct MockGraph { size_t nodes; };
struct MockGraphExec { size_t nodes; };
struct MockPlan { int dummy; };
struct MockInfo { void* stream = nullptr; };

static std::set<void*> g_streams, g_events, g_graphs, g_execs, g_infos;
static std::map<int, Capture> g_caps;
static int g_next_cap = 1;
static long g_ops = 0, g_memset_in_capture = 0;

static MockStream* S(hipStream_t s, const char* where) {
    if (!s) FAIL("%s on the null stream", where);
    if (!g_streams.count(s)) FAIL("%s on an invalid stream %p", where, (void*)s);
    return s;
}
static MockEvent* E(hipEvent_t e, const char* where) {
    if (!g_events.count(e)) FAIL("%s with an invalid event %p", where, (void*)e);
    return e;
}
static void node(MockStream* s) {
    ++g_ops;
    if (!s->capture) return;
    Capture& c = g_caps[s->capture];
    if (!c.open) FAIL("stream left in a capture that has ended");
    c.deps.push_back(s->frontier);
    s->frontier = {(int)c.deps.size() - 1};
}

// every launcher stub records its launch here
void mock_stream_op(MockStream* s, const char* what) { node(S(s, what)); }

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    *s = new MockStream();
    g_streams.insert(*s);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    if (S(s, "hipStreamDestroy")->capture) FAIL("destroying a capturing stream");
    g_streams.erase(s);
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    if (S(s, "hipStreamSynchronize")->capture) FAIL("synchronising a capturing stream");
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
    MockStream* st = S(s, "hipStreamWaitEvent");
    MockEvent* ev = E(e, "hipStreamWaitEvent");
    if (!ev->recorded) FAIL("wait on an event never recorded");
    if (ev->capture) {
        Capture& c = g_caps[ev->capture];
        if (!c.open) FAIL("wait on an event recorded in a capture that has ended");
        if (st->capture && st->capture != ev->capture) FAIL("a wait that joins two captures");
        if (!st->capture) {
            st->capture = ev->capture;
            st->frontier.clear();
        }
        st->frontier.insert(st->frontier.end(), ev->nodes.begin(), ev->nodes.end());
    } else if (st->capture) {
        FAIL("a capturing stream waits on an event recorded outside the capture");
    }
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    MockStream* st = S(s, "hipStreamBeginCapture");
    if (st->capture) FAIL("capture begun on a capturing stream");
    const int id = g_next_cap++;
    g_caps[id] = Capture{st, {}, true};
    st->capture = id;
    st->frontier.clear();
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
    MockStream* st = S(s, "hipStreamEndCapture");
    const int cid = st->capture;
    if (!cid) FAIL("end of capture on a stream that is not capturing");
    Capture& c = g_caps[cid];
    if (c.origin != st) FAIL("end of capture on a stream that did not begin it");
    std::vector<char> anc(c.deps.size(), 0);   // ancestors of the origin's last nodes
    std::vector<int> todo = st->frontier;
    while (!todo.empty()) {
        const int n = todo.back();
        todo.pop_back();
        if (anc[n]) continue;
        anc[n] = 1;
        for (int d : c.deps[n]) todo.push_back(d);
    }
    for (void* p : g_streams) {
        MockStream* o = (MockStream*)p;
        if (o->capture != cid) continue;
        for (int n : o->frontier)
            if (!anc[n]) FAIL("a forked stream did not join back before the end of the capture");
        o->capture = 0;
        o->frontier.clear();
    }
    for (size_t n = 0; n < anc.size(); ++n)
        if (!anc[n]) FAIL("captured node %zu is not joined into the origin stream", n);
    c.open = false;
    *g = new MockGraph{c.deps.size()};
    g_graphs.insert(*g);
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
    *e = new MockEvent();
    g_events.insert(*e);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned f) {
    hipEventCreate(e);
    (*e)->flags = f;
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    E(e, "hipEventDestroy");
    g_events.erase(e);
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    MockEvent* ev = E(e, "hipEventRecord");
    MockStream* st = S(s, "hipEventRecord");
    ev->recorded = true;
    ev->capture = st->capture;
    ev->nodes = st->frontier;
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    MockEvent* ev = E(e, "hipEventSynchronize");
    if (!ev->recorded) FAIL("synchronising on an event never recorded");
    if (ev->capture && g_caps[ev->capture].open) FAIL("synchronising on an event inside a capture");
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float* t, hipEvent_t a, hipEvent_t b) {
    if (!E(a, "hipEventElapsedTime")->recorded || !E(b, "hipEventElapsedTime")->recorded)
        FAIL("elapsed time of an event never recorded");
    if ((a->flags | b->flags) & hipEventDisableTiming) FAIL("elapsed time of a non-timing event");
    *t = 1.0f;
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
    if (!g_graphs.count(g)) FAIL("instantiating an invalid graph");
    *x = new MockGraphExec{g->nodes};
    g_execs.insert(*x);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
    if (!g_execs.count(x)) FAIL("launching an invalid graph");
    node(S(s, "hipGraphLaunch"));
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    if (!g_graphs.count(g)) FAIL("destroying an invalid graph");
    g_graphs.erase(g);
    delete g;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
    if (!g_execs.count(x)) FAIL("destroying an invalid graph exec");
    g_execs.erase(x);
    delete x;
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t st) {
    node(S(st, "hipMemcpyAsync"));
    if (n) std::memmove(d, s, n);
    return hipSuccess;
}
hipError_t hipMemcpy2DAsync(void* d, size_t dp, const void* s, size_t sp, size_t w, size_t h, hipMemcpyKind,
                            hipStream_t st) {
    node(S(st, "hipMemcpy2DAsync"));
    for (size_t r = 0; r < h; ++r) std::memmove((char*)d + r * dp, (const char*)s + r * sp, w);
    return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
    if (n) std::memmove(d, s, n);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t s) {
    MockStream* st = S(s, "hipMemsetAsync");
    if (st->capture) ++g_memset_in_capture;
    node(st);
    std::memset(d, v, n);
    return hipSuccess;
}
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 256; return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "mock error"; }

rocfft_status rocfft_setup() { return rocfft_status_success; }
rocfft_status rocfft_plan_create(rocfft_plan* p, rocfft_result_placement, rocfft_transform_type, rocfft_precision,
                                 size_t, const size_t*, size_t, const rocfft_plan_description) {
    *p = new MockPlan{0};
    return rocfft_status_success;
}
rocfft_status rocfft_plan_destroy(rocfft_plan p) { delete p; return rocfft_status_success; }
rocfft_status rocfft_plan_get_work_buffer_size(const rocfft_plan, size_t* n) { *n = 0; return rocfft_status_success; }
rocfft_status rocfft_execution_info_create(rocfft_execution_info* i) {
    *i = new MockInfo();
    g_infos.insert(*i);
    return rocfft_status_success;
}
rocfft_status rocfft_execution_info_destroy(rocfft_execution_info i) {
    if (!g_infos.count(i)) FAIL("destroying an invalid execution info");
    g_infos.erase(i);
    delete i;
    return rocfft_status_success;
}
rocfft_status rocfft_execution_info_set_stream(rocfft_execution_info i, void* s) {
    if (!g_infos.count(i)) FAIL("invalid execution info");
    S((hipStream_t)s, "rocfft_execution_info_set_stream");
    i->stream = s;
    return rocfft_status_success;
}
rocfft_status rocfft_execution_info_set_work_buffer(rocfft_execution_info, void*, size_t) { return rocfft_status_success; }
rocfft_status rocfft_execute(const rocfft_plan, void**, void**, rocfft_execution_info i) {
    if (!g_infos.count(i)) FAIL("invalid execution info");
    if (!i->stream) FAIL("rocfft_execute without a stream");
    node(S((hipStream_t)i->stream, "rocfft_execute"));
    return rocfft_status_success;
}

// rocBLAS: handles checked, every GEMM recorded as a node on the handle's stream
#include <rocblas/rocblas.h>
struct MockBlas { MockStream* stream = nullptr; };
static std::set<void*> g_blas;
rocblas_status rocblas_create_handle(rocblas_handle* h) {
    *h = new MockBlas();
    g_blas.insert(*h);
    return rocblas_status_success;
}
rocblas_status rocblas_destroy_handle(rocblas_handle h) {
    if (!g_blas.count(h)) FAIL("destroying an invalid rocBLAS handle");
    g_blas.erase(h);
    delete h;
    return rocblas_status_success;
}
rocblas_status rocblas_set_stream(rocblas_handle h, MockStream* s) {
    if (!g_blas.count(h)) FAIL("invalid rocBLAS handle");
    h->stream = S(s, "rocblas_set_stream");
    return rocblas_status_success;
}
static rocblas_status gemm_node(rocblas_handle h, int m, int n, int k, int lda, int ldb, int ldc) {
    if (!g_blas.count(h)) FAIL("invalid rocBLAS handle");
    if (m < 0 || n < 0 || k < 0 || lda < 1 || ldb < 1 || ldc < m) FAIL("gemm sizes");
    node(S(h->stream, "rocblas gemm"));
    return rocblas_status_success;
}
rocblas_status rocblas_cgemm(rocblas_handle h, rocblas_operation, rocblas_operation, rocblas_int m, rocblas_int n,
                             rocblas_int k, const rocblas_float_complex*, const rocblas_float_complex*, rocblas_int lda,
                             const rocblas_float_complex*, rocblas_int ldb, const rocblas_float_complex*,
                             rocblas_float_complex*, rocblas_int ldc) {
    return gemm_node(h, m, n, k, lda, ldb, ldc);
}
rocblas_status rocblas_zgemm(rocblas_handle h, rocblas_operation, rocblas_operation, rocblas_int m, rocblas_int n,
                             rocblas_int k, const rocblas_double_complex*, const rocblas_double_complex*,
                             rocblas_int lda, const rocblas_double_complex*, rocblas_int ldb,
                             const rocblas_double_complex*, rocblas_double_complex*, rocblas_int ldc) {
    return gemm_node(h, m, n, k, lda, ldb, ldc);
}

rocblas_status rocblas_cgemm_strided_batched(rocblas_handle h, rocblas_operation, rocblas_operation, rocblas_int m,
                                             rocblas_int n, rocblas_int k, const rocblas_float_complex*,
                                             const rocblas_float_complex*, rocblas_int lda, rocblas_stride,
                                             const rocblas_float_complex*, rocblas_int ldb, rocblas_stride,
                                             const rocblas_float_complex*, rocblas_float_complex*, rocblas_int ldc,
                                             rocblas_stride, rocblas_int batch) {
    if (batch < 1) FAIL("batch count");
    return gemm_node(h, m, n, k, lda, ldb, ldc);
}
rocblas_status rocblas_zgemm_strided_batched(rocblas_handle h, rocblas_operation, rocblas_operation, rocblas_int m,
                                             rocblas_int n, rocblas_int k, const rocblas_double_complex*,
                                             const rocblas_double_complex*, rocblas_int lda, rocblas_stride,
                                             const rocblas_double_complex*, rocblas_int ldb, rocblas_stride,
                                             const rocblas_double_complex*, rocblas_double_complex*, rocblas_int ldc,
                                             rocblas_stride, rocblas_int batch) {
    if (batch < 1) FAIL("batch count");
    return gemm_node(h, m, n, k, lda, ldb, ldc);
}

extern "C" void* mock_new_stream() {
    hipStream_t s;
    hipStreamCreateWithFlags(&s, 0);
    return s;
}
extern "C" long mock_ops() { return g_ops; }
extern "C" long mock_memsets_in_capture() { return g_memset_in_capture; }
// handles still alive (streams include the caller's own)
extern "C" long mock_live_handles() {
    return (long)(g_streams.size() + g_events.size() + g_graphs.size() + g_execs.size() + g_infos.size() +
                  g_blas.size());
}
