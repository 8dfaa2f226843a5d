// CPU emulation runtime for the host-emulation tests: work-items of a
// workgroup as cooperative coroutines, barriers and wave
// operations (stack switching), streams / events / stream capture (captured work is recorded
// and replayed by hipGraphLaunch, validated as a dependency graph like the
// stand-in of tests/host_mock), memory operations on host memory, and a
// rocFFT stand-in that evaluates the real 3-D transforms by direct separable
// DFTs.  Misuse aborts with a message and a backtrace.
#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <cxxabi.h>
#include <dlfcn.h>
#include <execinfo.h>
#include <sys/mman.h>

#include <chrono>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <map>
#include <memory>
#include <set>
#include <vector>

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define EMU_ASAN 1
#include <sanitizer/asan_interface.h>
#endif
#endif

#define FAIL(...)                                                  \
    do {                                                           \
        std::fprintf(stderr, "EMU ERROR: " __VA_ARGS__);           \
        std::fprintf(stderr, "\n");                                \
        void* bt_[40];                                             \
        backtrace_symbols_fd(bt_, backtrace(bt_, 40), 2);          \
        std::abort();                                              \
    } while (0)

namespace emu {

dim3 threadIdx_v, blockIdx_v, blockDim_v, gridDim_v;

// ------------------------------------------------------------ work-items
// Stack switch between the scheduler and the work-items (x86-64 System V):
// saves the callee-saved registers, MXCSR and the x87 control word on the
// current stack, stores the stack pointer in *from and continues on `to`.
extern "C" void emu_switch(void** from, void* to);
asm(R"(
    .text
    .globl emu_switch
    .type emu_switch, @function
emu_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    subq $8, %rsp
    stmxcsr (%rsp)
    fnstcw 4(%rsp)
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    ldmxcsr (%rsp)
    fldcw 4(%rsp)
    addq $8, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
    .size emu_switch, .-emu_switch
)");

enum class St { Ready, Barrier, Wave, Done };
struct Lane {
    void* sp = nullptr;
    St st = St::Done;
    WaveOp op{};
    int param = 0, width = 64;
    unsigned char in[64];
    size_t in_bytes = 0;
    void* out = nullptr;
    size_t out_bytes = 0;
};

constexpr size_t STACK = 64 * 1024;
constexpr int MAX_LANES = 1024;
static std::vector<Lane> g_lanes(MAX_LANES);
static char* g_stacks = nullptr;
static void* g_sched_sp = nullptr;
static int g_cur = -1, g_nlanes = 0;
static void (*g_thunk)(void*) = nullptr;
static void* g_arg = nullptr;
static std::vector<unsigned char> g_dyn;

static void to_sched() { emu_switch(&g_lanes[g_cur].sp, g_sched_sp); }

[[noreturn]] static void lane_entry() {
    g_thunk(g_arg);
    g_lanes[g_cur].st = St::Done;
    emu_switch(&g_lanes[g_cur].sp, g_sched_sp);
    std::abort();   // a finished work-item is never resumed
}

static void set_ids(int i) {
    threadIdx_v = dim3(i % blockDim_v.x, (i / blockDim_v.x) % blockDim_v.y, i / (blockDim_v.x * blockDim_v.y));
}

static void resume(int i) {
    g_cur = i;
    set_ids(i);
    emu_switch(&g_sched_sp, g_lanes[i].sp);
    g_cur = -1;
}

// a fresh work-item stack whose first switch "returns" into lane_entry
static void* fresh_stack(int i) {
    char* top = g_stacks + (size_t)(i + 1) * STACK;
    uint64_t* p = reinterpret_cast<uint64_t*>(top - 16);      // 16-byte aligned return slot
    p[0] = reinterpret_cast<uint64_t>(&lane_entry);
    p[1] = 0;
    uint64_t* q = p - 7;                                       // rbp rbx r12 r13 r14 r15, then csr
    for (int k = 1; k <= 6; ++k) q[k] = 0;
    const uint32_t mxcsr = 0x1F80;
    const uint16_t fpcw = 0x037F;
    std::memcpy(reinterpret_cast<char*>(q), &mxcsr, 4);
    std::memcpy(reinterpret_cast<char*>(q) + 4, &fpcw, 2);
    return q;
}

void syncthreads() {
    if (g_cur < 0) FAIL("__syncthreads outside a kernel");
    g_lanes[g_cur].st = St::Barrier;
    to_sched();
}

void wave_op(WaveOp op, const void* in, size_t in_bytes, void* out, size_t out_bytes, int param, int width) {
    if (g_cur < 0) FAIL("wave operation outside a kernel");
    if (in_bytes > sizeof(Lane::in)) FAIL("wave operand too large");
    Lane& l = g_lanes[g_cur];
    l.op = op;
    l.param = param;
    l.width = width;
    std::memcpy(l.in, in, in_bytes);
    l.in_bytes = in_bytes;
    l.out = out;
    l.out_bytes = out_bytes;
    l.st = St::Wave;
    to_sched();
}

void* dyn_lds() { return g_dyn.data(); }

static float bf(__bf16 v) { return (float)v; }

static void resolve_wave(int w0, int w1) {
    const Lane& first = g_lanes[w0];
    int lead = -1;
    for (int i = w0; i < w1; ++i)
        if (g_lanes[i].st == St::Wave) { lead = i; break; }
    (void)first;
    const WaveOp op = g_lanes[lead].op;
    for (int i = w0; i < w1; ++i)
        if (g_lanes[i].st == St::Wave && (g_lanes[i].op != op || g_lanes[i].param != g_lanes[lead].param))
            FAIL("lanes of one wave are at different wave operations");
    auto live = [&](int i) { return i < w1 && g_lanes[i].st == St::Wave; };
    switch (op) {
    case WaveOp::ShflXor:
    case WaveOp::ShflUp:
        for (int i = w0; i < w1; ++i) {
            Lane& l = g_lanes[i];
            if (l.st != St::Wave) continue;
            const int lane = i - w0, w = l.width, seg = lane - lane % w;
            int src;
            if (op == WaveOp::ShflXor) src = lane ^ l.param;
            else src = (lane - l.param >= seg) ? lane - l.param : lane;
            if (src < seg || src >= seg + w) src = lane;
            if (live(w0 + src)) std::memcpy(l.out, g_lanes[w0 + src].in, l.out_bytes);
            else std::memset(l.out, 0, l.out_bytes);
        }
        break;
    case WaveOp::Ballot: {
        unsigned long long m = 0;
        for (int i = w0; i < w1; ++i)
            if (live(i)) {
                int p;
                std::memcpy(&p, g_lanes[i].in, sizeof(int));
                if (p) m |= 1ull << (i - w0);
            }
        for (int i = w0; i < w1; ++i)
            if (live(i)) std::memcpy(g_lanes[i].out, &m, sizeof(m));
        break;
    }
    case WaveOp::Mfma16x16x32Bf16: {
        // lane l: A row l%16, k = 8(l/16)..+7; B column l%16, same k;
        // D column l%16, rows 4(l/16)..+3
        struct In { emu_bf16x8 a, b; emu_f32x4 c; };
        float A[16][32] = {}, B[32][16] = {}, C[16][16] = {};
        for (int i = w0; i < w1; ++i) {
            if (!live(i)) continue;
            In v;
            std::memcpy(&v, g_lanes[i].in, sizeof(In));
            const int l = i - w0, r = l % 16, kb = 8 * (l / 16);
            for (int k = 0; k < 8; ++k) {
                A[r][kb + k] = bf(v.a[k]);
                B[kb + k][r] = bf(v.b[k]);
            }
            for (int j = 0; j < 4; ++j) C[4 * (l / 16) + j][r] = v.c[j];
        }
        for (int i = w0; i < w1; ++i) {
            if (!live(i)) continue;
            const int l = i - w0, col = l % 16;
            emu_f32x4 d;
            for (int j = 0; j < 4; ++j) {
                const int row = 4 * (l / 16) + j;
                float s = C[row][col];
                for (int k = 0; k < 32; ++k) s += A[row][k] * B[k][col];
                d[j] = s;
            }
            std::memcpy(g_lanes[i].out, &d, sizeof(d));
        }
        break;
    }
    }
    for (int i = w0; i < w1; ++i)
        if (g_lanes[i].st == St::Wave) g_lanes[i].st = St::Ready;
}

static void run_block() {
    const int n = g_nlanes;
    for (int i = 0; i < n; ++i) {
        g_lanes[i].sp = fresh_stack(i);
        g_lanes[i].st = St::Ready;
    }
    for (;;) {
        bool ran = false;
        for (int i = 0; i < n; ++i)
            if (g_lanes[i].st == St::Ready) {
                resume(i);
                ran = true;
            }
        int live = 0, bar = 0;
        for (int i = 0; i < n; ++i) {
            if (g_lanes[i].st != St::Done) ++live;
            if (g_lanes[i].st == St::Barrier) ++bar;
        }
        if (live == 0) break;
        bool released = false;
        if (bar == live) {
            for (int i = 0; i < n; ++i) g_lanes[i].st = St::Ready;
            released = true;
        } else {
            for (int w0 = 0; w0 < n; w0 += 64) {
                const int w1 = std::min(n, w0 + 64);
                int lw = 0, at = 0;
                for (int i = w0; i < w1; ++i) {
                    if (g_lanes[i].st != St::Done) ++lw;
                    if (g_lanes[i].st == St::Wave) ++at;
                }
                if (lw > 0 && at == lw) {
                    resolve_wave(w0, w1);
                    released = true;
                }
            }
        }
        if (!ran && !released) {
            int w = 0, b = 0, d = 0;
            for (int i = 0; i < n; ++i) {
                w += g_lanes[i].st == St::Wave;
                b += g_lanes[i].st == St::Barrier;
                d += g_lanes[i].st == St::Done;
            }
            FAIL("deadlock in a workgroup: %d at barriers, %d at wave operations, %d finished of %d", b, w, d, n);
        }
    }
}

// EMU_PROFILE=1: time spent per kernel, printed at exit
struct Prof { double s = 0; long n = 0; long lanes = 0; };
static std::map<void*, Prof>* g_prof = nullptr;
static void prof_dump() {
    std::vector<std::pair<double, std::string>> rows;
    for (auto& kv : *g_prof) {
        Dl_info di{};
        std::string name = "?";
        if (dladdr(kv.first, &di) && di.dli_sname) {
            int st = 0;
            char* d = abi::__cxa_demangle(di.dli_sname, nullptr, nullptr, &st);
            name = d ? d : di.dli_sname;
            std::free(d);
        }
        const size_t k = name.find("[](auto...) {");
        if (name.size() > 160) name = name.substr(0, 160);
        char buf[64];
        std::snprintf(buf, sizeof buf, "%8.2f s %6ld launches %10ld lanes  ", kv.second.s, kv.second.n, kv.second.lanes);
        rows.push_back({kv.second.s, std::string(buf) + name});
        (void)k;
    }
    std::sort(rows.rbegin(), rows.rend());
    for (auto& r : rows) std::fprintf(stderr, "%s\n", r.second.c_str());
}

static void run_launch(dim3 grid, dim3 block, size_t lds, void (*thunk)(void*), void* arg) {
    static const bool prof = std::getenv("EMU_PROFILE") != nullptr;
    if (prof && !g_prof) {
        g_prof = new std::map<void*, Prof>();
        std::atexit(prof_dump);
    }
    const auto t0 = std::chrono::steady_clock::now();
    const long nthreads = (long)block.x * block.y * block.z;
    if (nthreads < 1 || nthreads > MAX_LANES) FAIL("workgroup of %ld work-items", nthreads);
    if (lds > 160 * 1024) FAIL("dynamic LDS of %zu bytes", lds);
    if (!g_stacks) {
        g_stacks = (char*)mmap(nullptr, STACK * MAX_LANES, PROT_READ | PROT_WRITE,
                               MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
        if (g_stacks == MAP_FAILED) FAIL("mmap of the work-item stacks");
    }
    g_dyn.assign(lds + 16, 0xA5);   // uninitialised LDS reads see a fixed pattern
    g_thunk = thunk;
    g_arg = arg;
    blockDim_v = block;
    gridDim_v = grid;
    g_nlanes = (int)nthreads;
    for (unsigned z = 0; z < grid.z; ++z)
        for (unsigned y = 0; y < grid.y; ++y)
            for (unsigned x = 0; x < grid.x; ++x) {
                blockIdx_v = dim3(x, y, z);
                run_block();
            }
    if (prof) {
        Prof& p = (*g_prof)[(void*)thunk];
        p.s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        p.n += 1;
        p.lanes += (long)grid.x * grid.y * grid.z * nthreads;
    }
}

void poison(void* p, size_t n) {
#ifdef EMU_ASAN
    ASAN_POISON_MEMORY_REGION(p, n);
#else
    (void)p;
    (void)n;
#endif
}

}  // namespace emu

// ------------------------------------------------------------ streams, capture
struct Capture {
    MockStream* origin;
    std::vector<std::vector<int>> deps;
    std::vector<std::function<void()>> ops;
    bool open;
};
struct MockStream { int capture = 0; std::vector<int> frontier; };
struct MockEvent { bool recorded = false; int capture = 0; std::vector<int> nodes; unsigned flags = 0; };
struct MockGraph { std::vector<std::function<void()>> ops; };
struct MockGraphExec { std::vector<std::function<void()>> ops; };
struct MockPlan { bool forward; size_t n[3]; };
struct MockInfo { void* stream = nullptr; };

static std::set<void*> g_streams, g_events, g_graphs, g_execs, g_infos;
static std::map<int, Capture> g_caps;
static int g_next_cap = 1;
static long g_memset_in_capture = 0, g_launches = 0;

static MockStream* S(hipStream_t s, const char* where) {
    if (!s) FAIL("%s on the null stream", where);
    if (!g_streams.count(s)) FAIL("%s on an invalid stream %p", where, (void*)s);
    return s;
}
static MockEvent* E(hipEvent_t e, const char* where) {
    if (!g_events.count(e)) FAIL("%s with an invalid event %p", where, (void*)e);
    return e;
}
// run `op` now, or record it into the capture the stream belongs to
static void submit(MockStream* s, std::function<void()> op) {
    if (!s->capture) {
        op();
        return;
    }
    Capture& c = g_caps[s->capture];
    if (!c.open) FAIL("stream left in a capture that has ended");
    c.deps.push_back(s->frontier);
    c.ops.push_back(std::move(op));
    s->frontier = {(int)c.deps.size() - 1};
}

void emu::launch_impl(dim3 grid, dim3 block, size_t lds, hipStream_t s, void (*thunk)(void*), void* arg,
                      void (*destroy)(void*)) {
    ++g_launches;
    std::shared_ptr<void> keep(arg, destroy);
    auto op = [grid, block, lds, thunk, keep]() { emu::run_launch(grid, block, lds, thunk, keep.get()); };
    if (!s) op();
    else submit(S(s, "kernel launch"), op);
}

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
    g_caps[id] = Capture{st, {}, {}, true};
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
    std::vector<char> anc(c.deps.size(), 0);
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
    *g = new MockGraph{std::move(c.ops)};
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
    *x = new MockGraphExec{g->ops};
    g_execs.insert(*x);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
    if (!g_execs.count(x)) FAIL("launching an invalid graph");
    MockGraphExec* ex = x;
    submit(S(s, "hipGraphLaunch"), [ex]() {
        for (auto& op : ex->ops) op();
    });
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
    submit(S(st, "hipMemcpyAsync"), [d, s, n]() { if (n) std::memmove(d, s, n); });
    return hipSuccess;
}
hipError_t hipMemcpy2DAsync(void* d, size_t dp, const void* s, size_t sp, size_t w, size_t h, hipMemcpyKind,
                            hipStream_t st) {
    submit(S(st, "hipMemcpy2DAsync"), [=]() {
        for (size_t r = 0; r < h; ++r) std::memmove((char*)d + r * dp, (const char*)s + r * sp, w);
    });
    return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
    if (n) std::memmove(d, s, n);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t s) {
    MockStream* st = S(s, "hipMemsetAsync");
    if (st->capture) ++g_memset_in_capture;
    submit(st, [d, v, n]() { std::memset(d, v, n); });
    return hipSuccess;
}
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
// a small device: the persistent launches get few workgroups, which keeps the emulation fast
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 4; return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "emulated error"; }

// ------------------------------------------------------------ rocFFT by direct DFTs
using cd = std::complex<double>;
static void dft_axis(cd* a, size_t n, size_t stride, size_t count, size_t jump, int sign) {
    std::vector<cd> w(n), tmp(n);
    for (size_t k = 0; k < n; ++k) w[k] = std::polar(1.0, sign * 2.0 * M_PI * (double)k / (double)n);
    for (size_t c = 0; c < count; ++c) {
        cd* p = a + c * jump;
        for (size_t k = 0; k < n; ++k) {
            cd s = 0.0;
            for (size_t j = 0; j < n; ++j) s += p[j * stride] * w[(j * k) % n];
            tmp[k] = s;
        }
        for (size_t k = 0; k < n; ++k) p[k * stride] = tmp[k];
    }
}
static void exec_plan(const MockPlan* p, void* in, void* out) {
    const size_t nx = p->n[0], ny = p->n[1], nz = p->n[2], nh = nx / 2 + 1;
    std::vector<cd> h(nz * ny * nh);
    if (p->forward) {
        const double* x = (const double*)in;
        std::vector<cd> w(nx);
        for (size_t k = 0; k < nx; ++k) w[k] = std::polar(1.0, -2.0 * M_PI * (double)k / (double)nx);
        for (size_t r = 0; r < nz * ny; ++r)
            for (size_t k = 0; k < nh; ++k) {
                cd s = 0.0;
                for (size_t j = 0; j < nx; ++j) s += x[r * nx + j] * w[(j * k) % nx];
                h[r * nh + k] = s;
            }
        for (size_t z = 0; z < nz; ++z) dft_axis(h.data() + z * ny * nh, ny, nh, nh, 1, -1);
        dft_axis(h.data(), nz, ny * nh, ny * nh, 1, -1);
        std::memcpy(out, h.data(), h.size() * sizeof(cd));
    } else {
        std::memcpy(h.data(), in, h.size() * sizeof(cd));
        dft_axis(h.data(), nz, ny * nh, ny * nh, 1, +1);
        for (size_t z = 0; z < nz; ++z) dft_axis(h.data() + z * ny * nh, ny, nh, nh, 1, +1);
        double* x = (double*)out;
        for (size_t r = 0; r < nz * ny; ++r)
            for (size_t j = 0; j < nx; ++j) {
                double s = h[r * nh].real();
                for (size_t k = 1; k < nh; ++k) {
                    const cd e = std::polar(1.0, 2.0 * M_PI * (double)((j * k) % nx) / (double)nx);
                    const double t = (h[r * nh + k] * e).real();
                    s += (nx % 2 == 0 && k == nx / 2) ? t : 2.0 * t;
                }
                x[r * nx + j] = s;
            }
    }
}

rocfft_status rocfft_setup() { return rocfft_status_success; }
rocfft_status rocfft_plan_create(rocfft_plan* p, rocfft_result_placement pl, rocfft_transform_type t,
                                 rocfft_precision prec, size_t dims, const size_t* len, size_t batch,
                                 const rocfft_plan_description) {
    if (pl != rocfft_placement_notinplace || prec != rocfft_precision_double || dims != 3 || batch != 1)
        FAIL("unsupported FFT plan");
    if (t != rocfft_transform_type_real_forward && t != rocfft_transform_type_real_inverse)
        FAIL("unsupported FFT type");
    *p = new MockPlan{t == rocfft_transform_type_real_forward, {len[0], len[1], len[2]}};
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
rocfft_status rocfft_execute(const rocfft_plan p, void** in, void** out, rocfft_execution_info i) {
    if (!g_infos.count(i)) FAIL("invalid execution info");
    if (!i->stream) FAIL("rocfft_execute without a stream");
    void* a = in[0];
    void* b = out[0];
    const MockPlan* plan = p;
    submit(S((hipStream_t)i->stream, "rocfft_execute"), [plan, a, b]() { exec_plan(plan, a, b); });
    return rocfft_status_success;
}

extern "C" void* mock_new_stream() {
    hipStream_t s;
    hipStreamCreateWithFlags(&s, 0);
    return s;
}
extern "C" long mock_memsets_in_capture() { return g_memset_in_capture; }
extern "C" long mock_launches() { return g_launches; }
static std::set<void*> g_blas;
extern "C" long mock_live_handles() {
    return (long)(g_streams.size() + g_events.size() + g_graphs.size() + g_execs.size() + g_infos.size() +
                  g_blas.size());
}

// ------------------------------------------------------------ rocBLAS by direct loops
#include <rocblas/rocblas.h>
struct MockBlas { MockStream* stream = nullptr; };
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
    S(s, "rocblas_set_stream");
    h->stream = s;
    return rocblas_status_success;
}
template <class R>
static rocblas_status gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
                           std::complex<R> alpha, const std::complex<R>* A, int lda, const std::complex<R>* B, int ldb,
                           std::complex<R> beta, std::complex<R>* C, int ldc) {
    if (!g_blas.count(h)) FAIL("invalid rocBLAS handle");
    if (ta == rocblas_operation_transpose || tb == rocblas_operation_transpose) FAIL("unexpected gemm operation");
    const bool ca = ta == rocblas_operation_conjugate_transpose, cb = tb == rocblas_operation_conjugate_transpose;
    if (m < 0 || n < 0 || k < 0 || ldc < std::max(1, m) || lda < std::max(1, ca ? k : m) || ldb < std::max(1, cb ? n : k))
        FAIL("gemm sizes: m %d n %d k %d lda %d ldb %d ldc %d", m, n, k, lda, ldb, ldc);
    submit(S(h->stream, "rocblas gemm"), [=]() {
        std::vector<std::complex<R>> col(m);
        for (int j = 0; j < n; ++j) {
            std::fill(col.begin(), col.end(), std::complex<R>(0));
            for (int p = 0; p < k; ++p) {
                const std::complex<R> b = cb ? std::conj(B[j + (size_t)p * ldb]) : B[p + (size_t)j * ldb];
                for (int i = 0; i < m; ++i) {
                    const std::complex<R> a = ca ? std::conj(A[p + (size_t)i * lda]) : A[i + (size_t)p * lda];
                    col[i] += a * b;
                }
            }
            for (int i = 0; i < m; ++i) {
                std::complex<R>& c = C[i + (size_t)j * ldc];
                c = alpha * col[i] + (beta == std::complex<R>(0) ? std::complex<R>(0) : beta * c);
            }
        }
    });
    return rocblas_status_success;
}
rocblas_status rocblas_cgemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, rocblas_int m, rocblas_int n,
                             rocblas_int k, const rocblas_float_complex* alpha, const rocblas_float_complex* A,
                             rocblas_int lda, const rocblas_float_complex* B, rocblas_int ldb,
                             const rocblas_float_complex* beta, rocblas_float_complex* C, rocblas_int ldc) {
    using c = std::complex<float>;
    return gemm<float>(h, ta, tb, m, n, k, c(alpha->x, alpha->y), reinterpret_cast<const c*>(A), lda,
                       reinterpret_cast<const c*>(B), ldb, c(beta->x, beta->y), reinterpret_cast<c*>(C), ldc);
}
rocblas_status rocblas_zgemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, rocblas_int m, rocblas_int n,
                             rocblas_int k, const rocblas_double_complex* alpha, const rocblas_double_complex* A,
                             rocblas_int lda, const rocblas_double_complex* B, rocblas_int ldb,
                             const rocblas_double_complex* beta, rocblas_double_complex* C, rocblas_int ldc) {
    using c = std::complex<double>;
    return gemm<double>(h, ta, tb, m, n, k, c(alpha->x, alpha->y), reinterpret_cast<const c*>(A), lda,
                        reinterpret_cast<const c*>(B), ldb, c(beta->x, beta->y), reinterpret_cast<c*>(C), ldc);
}
rocblas_status rocblas_cgemm_strided_batched(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, rocblas_int m,
                                             rocblas_int n, rocblas_int k, const rocblas_float_complex* alpha,
                                             const rocblas_float_complex* A, rocblas_int lda, rocblas_stride sa,
                                             const rocblas_float_complex* B, rocblas_int ldb, rocblas_stride sb,
                                             const rocblas_float_complex* beta, rocblas_float_complex* C,
                                             rocblas_int ldc, rocblas_stride sc, rocblas_int batch) {
    if (batch < 1) FAIL("batch count %d", batch);
    for (int b = 0; b < batch; ++b) {
        const rocblas_status st =
            rocblas_cgemm(h, ta, tb, m, n, k, alpha, A + b * sa, lda, B + b * sb, ldb, beta, C + b * sc, ldc);
        if (st != rocblas_status_success) return st;
    }
    return rocblas_status_success;
}
rocblas_status rocblas_zgemm_strided_batched(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, rocblas_int m,
                                             rocblas_int n, rocblas_int k, const rocblas_double_complex* alpha,
                                             const rocblas_double_complex* A, rocblas_int lda, rocblas_stride sa,
                                             const rocblas_double_complex* B, rocblas_int ldb, rocblas_stride sb,
                                             const rocblas_double_complex* beta, rocblas_double_complex* C,
                                             rocblas_int ldc, rocblas_stride sc, rocblas_int batch) {
    if (batch < 1) FAIL("batch count %d", batch);
    for (int b = 0; b < batch; ++b) {
        const rocblas_status st =
            rocblas_zgemm(h, ta, tb, m, n, k, alpha, A + b * sa, lda, B + b * sb, ldb, beta, C + b * sc, ldc);
        if (st != rocblas_status_success) return st;
    }
    return rocblas_status_success;
}
