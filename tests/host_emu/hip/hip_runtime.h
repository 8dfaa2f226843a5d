// CPU emulation of the HIP device language and runtime subset the library
// uses, for the host-emulation tests only.  Kernels become plain functions;
// emu::launch runs every work-item of a workgroup as a cooperative coroutine
// (barriers and wave operations switch between them), one workgroup after
// another.  LDS (__shared__) becomes static storage, shared by the
// work-items of the running workgroup.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <tuple>
#include <type_traits>
#include <utility>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))
// a __device__ variable is host storage here: its address is the symbol's own
#define HIP_SYMBOL(x) (&(x))

typedef enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorNotReady = 600,
    hipErrorUnknown = 999
} hipError_t;
struct MockStream;
struct MockEvent;
struct MockGraph;
struct MockGraphExec;
typedef MockStream* hipStream_t;
typedef MockEvent* hipEvent_t;
typedef MockGraph* hipGraph_t;
typedef MockGraphExec* hipGraphExec_t;
typedef void* hipGraphNode_t;
typedef enum { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
               hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 } hipMemcpyKind;
typedef enum { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1,
               hipStreamCaptureModeRelaxed = 2 } hipStreamCaptureMode;
typedef enum { hipDeviceAttributeMultiprocessorCount = 1 } hipDeviceAttribute_t;
#define hipStreamNonBlocking 1u
#define hipEventDisableTiming 2u
#define hipEventDefault 0u

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned x_ = 1, unsigned y_ = 1, unsigned z_ = 1) : x(x_), y(y_), z(z_) {}
};
struct float2 { float x, y; };
struct double2 { double x, y; };
struct int2 { int x, y; };
inline int2 make_int2(int a, int b) { return {a, b}; }
struct float4 { float x, y, z, w; };
inline float2 make_float2(float a, float b) { return {a, b}; }
inline double2 make_double2(double a, double b) { return {a, b}; }
inline float4 make_float4(float a, float b, float c, float d) { return {a, b, c, d}; }

using std::isfinite;
using std::isinf;
using std::isnan;
template <class A, class B>
inline typename std::common_type<A, B>::type min(A a, B b) { return a < b ? a : b; }
template <class A, class B>
inline typename std::common_type<A, B>::type max(A a, B b) { return a < b ? b : a; }

namespace emu {
extern dim3 threadIdx_v, blockIdx_v, blockDim_v, gridDim_v;
void syncthreads();
enum class WaveOp { ShflXor, ShflUp, Ballot, Mfma16x16x32Bf16 };
// one wave operation of the calling lane: in = its operand bytes; the
// result bytes (filled when every live lane of the wave has arrived) go to out
void wave_op(WaveOp op, const void* in, size_t in_bytes, void* out, size_t out_bytes, int param, int width);
void* dyn_lds();
// run (or, while the stream is captured, record) one kernel launch
void launch_impl(dim3 grid, dim3 block, size_t lds, hipStream_t s, void (*thunk)(void*), void* arg,
                 void (*destroy)(void*));
// ASan poisoning of workspace redzones
void poison(void* p, size_t n);

template <class F, class Tup>
struct Launch {
    F f;
    Tup args;
};
template <class F, class... A>
hipError_t launch(dim3 grid, dim3 block, size_t lds, hipStream_t s, F f, A... args) {
    using L = Launch<F, std::tuple<A...>>;
    L* l = new L{f, std::tuple<A...>(args...)};
    launch_impl(
        grid, block, lds, s, [](void* p) { L* q = static_cast<L*>(p); std::apply(q->f, q->args); }, l,
        [](void* p) { delete static_cast<L*>(p); });
    return hipSuccess;
}
template <class F, class... A>
hipError_t launch(dim3 grid, dim3 block, F f, A... args) {
    return launch(grid, block, 0, nullptr, f, args...);
}
}  // namespace emu

#define threadIdx emu::threadIdx_v
#define blockIdx emu::blockIdx_v
#define blockDim emu::blockDim_v
#define gridDim emu::gridDim_v
inline void __syncthreads() { emu::syncthreads(); }
inline void __threadfence() {}

template <class T>
inline T __shfl_xor(T v, int mask, int width = 64) {
    T r;
    emu::wave_op(emu::WaveOp::ShflXor, &v, sizeof(T), &r, sizeof(T), mask, width);
    return r;
}
template <class T>
inline T __shfl_up(T v, unsigned delta, int width = 64) {
    T r;
    emu::wave_op(emu::WaveOp::ShflUp, &v, sizeof(T), &r, sizeof(T), (int)delta, width);
    return r;
}
inline unsigned long long __ballot(int pred) {
    unsigned long long r;
    const int p = pred != 0;
    emu::wave_op(emu::WaveOp::Ballot, &p, sizeof(int), &r, sizeof(r), 0, 64);
    return r;
}
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
// work-items run one at a time between switch points, so read-modify-write is atomic
inline int atomicAdd(int* p, int v) { const int o = *p; *p = o + v; return o; }
inline int atomicExch(int* p, int v) { const int o = *p; *p = v; return o; }
inline int atomicOr(int* p, int v) { const int o = *p; *p = o | v; return o; }

typedef __bf16 emu_bf16x8 __attribute__((ext_vector_type(8)));
typedef float emu_f32x4 __attribute__((ext_vector_type(4)));
inline emu_f32x4 emu_mfma_f32_16x16x32_bf16(emu_bf16x8 a, emu_bf16x8 b, emu_f32x4 c) {
    struct { emu_bf16x8 a, b; emu_f32x4 c; } in{a, b, c};
    emu_f32x4 r;
    emu::wave_op(emu::WaveOp::Mfma16x16x32Bf16, &in, sizeof(in), &r, sizeof(r), 0, 64);
    return r;
}
#define __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, cbsz, abid, blgp) emu_mfma_f32_16x16x32_bf16(a, b, c)
// a wave barrier is a rendezvous of the wave's live lanes (any wave operation
// is one); waiting for memory counters has nothing to wait for here
inline void emu_wave_barrier() { (void)__ballot(1); }
#define __builtin_amdgcn_wave_barrier() emu_wave_barrier()
#define __builtin_amdgcn_s_waitcnt(x) ((void)0)

// runtime API (emu.cpp)
hipError_t hipStreamCreateWithFlags(hipStream_t*, unsigned);
hipError_t hipStreamDestroy(hipStream_t);
hipError_t hipStreamSynchronize(hipStream_t);
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned);
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode);
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t*);
hipError_t hipEventCreate(hipEvent_t*);
hipError_t hipEventCreateWithFlags(hipEvent_t*, unsigned);
hipError_t hipEventDestroy(hipEvent_t);
hipError_t hipEventRecord(hipEvent_t, hipStream_t);
hipError_t hipEventSynchronize(hipEvent_t);
hipError_t hipEventElapsedTime(float*, hipEvent_t, hipEvent_t);
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, hipGraphNode_t*, char*, size_t);
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t);
hipError_t hipGraphDestroy(hipGraph_t);
hipError_t hipGraphExecDestroy(hipGraphExec_t);
hipError_t hipMemcpyAsync(void*, const void*, size_t, hipMemcpyKind, hipStream_t);
hipError_t hipMemcpy2DAsync(void*, size_t, const void*, size_t, size_t, size_t, hipMemcpyKind, hipStream_t);
hipError_t hipMemcpy(void*, const void*, size_t, hipMemcpyKind);
hipError_t hipMemsetAsync(void*, int, size_t, hipStream_t);
hipError_t hipGetDevice(int*);
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) {
    *p = const_cast<void*>(sym);
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int*, hipDeviceAttribute_t, int);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t);
template <class F>
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, F, int block, size_t lds) {
    int by_lds = lds ? (int)((160 * 1024) / lds) : 8;
    int by_threads = 2048 / (block > 0 ? block : 1);
    *n = std::max(0, std::min(by_lds, by_threads));
    return hipSuccess;
}
