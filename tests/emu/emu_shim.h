// CPU emulation of the HIP subset used by libkfvol (checking tool, never shipped).
// Each GPU thread runs as a fiber; wave collectives (shuffles, readfirstlane, exec mask)
// and block barriers switch back to a per-block round-robin scheduler.
#pragma once
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

using std::max;
using std::min;

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static thread_local
#define __constant__
#define address_space(n)
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) ((const void*)&(x))

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct uint2 { uint32_t x, y; };
struct uint4 { uint32_t x, y, z, w; };
struct float2 { float x, y; };
struct float4 { float x, y, z, w; };
inline uint2 make_uint2(uint32_t a, uint32_t b) { return {a, b}; }
inline uint4 make_uint4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) { return {a, b, c, d}; }
inline float2 make_float2(float a, float b) { return {a, b}; }
inline float4 make_float4(float a, float b, float c, float d) { return {a, b, c, d}; }

extern thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;

// ---------------------------------------------------------------- collectives
namespace emu {
void yield_collective();            // end of this fiber's turn in the round
uint64_t* slots(int parity);        // per-thread 64-bit slots of the running block
int next_parity();                  // this thread's collective parity (toggles)
bool lane_done(unsigned tid);
void syncthreads();
void check_direct(const char* what);
}  // namespace emu

template <class T>
inline T emu_bcast_from(T v, int src_lane)
{
    emu::check_direct("collective");
    static_assert(sizeof(T) <= 8, "slot");
    const int p = emu::next_parity();
    uint64_t bits = 0;
    memcpy(&bits, &v, sizeof(T));
    emu::slots(p)[threadIdx.x] = bits;
    emu::yield_collective();
    const unsigned base = threadIdx.x & ~63u;
    T out;
    uint64_t got = emu::slots(p)[base + (unsigned)src_lane];
    memcpy(&out, &got, sizeof(T));
    return out;
}

inline uint64_t emu_exec_mask()
{
    emu::check_direct("exec");
    const unsigned base = threadIdx.x & ~63u;
    uint64_t m = 0;
    for (unsigned l = 0; l < 64; ++l)
        if (base + l < blockDim.x && !emu::lane_done(base + l)) m |= 1ull << l;
    return m;
}

inline int emu_first_lane()
{
    const uint64_t m = emu_exec_mask();
    return m ? __builtin_ctzll(m) : 0;
}

template <class T>
inline T __shfl_xor(T v, int mask, int width = 64)
{
    (void)width;
    const int lane = (int)(threadIdx.x & 63u);
    return emu_bcast_from(v, lane ^ mask);
}

template <class T>
inline T __shfl(T v, int src, int width = 64)
{
    (void)width;
    return emu_bcast_from(v, src & 63);
}

template <class T>
inline T __shfl_up(T v, unsigned delta, int width = 64)
{
    (void)width;
    const int lane = (int)(threadIdx.x & 63u);
    const int src = lane - (int)delta;
    return emu_bcast_from(v, src < 0 ? lane : src);
}

// like the builtin: takes and returns a signed 32-bit int
#define __builtin_amdgcn_readfirstlane(v) emu_readfirstlane((int)(v))
inline int emu_readfirstlane(int v)
{
    const int first = emu_first_lane();
    return emu_bcast_from(v, first);
}
#define __builtin_amdgcn_read_exec() emu_exec_mask()
inline uint32_t emu_mbcnt_lo(uint32_t m, uint32_t acc)
{
    const unsigned lane = threadIdx.x & 63u;
    const uint32_t below = lane >= 32 ? 0xFFFFFFFFu : ((1u << lane) - 1u);
    return acc + (uint32_t)__builtin_popcount(m & below);
}
inline uint32_t emu_mbcnt_hi(uint32_t m, uint32_t acc)
{
    const unsigned lane = threadIdx.x & 63u;
    const uint32_t below = lane < 32 ? 0u : ((1u << (lane - 32)) - 1u);
    return acc + (uint32_t)__builtin_popcount(m & below);
}
#define __builtin_amdgcn_mbcnt_lo(m, a) emu_mbcnt_lo(m, a)
#define __builtin_amdgcn_mbcnt_hi(m, a) emu_mbcnt_hi(m, a)

inline unsigned long long __ballot(int pred)
{
    emu::check_direct("ballot");
    const int p = emu::next_parity();
    emu::slots(p)[threadIdx.x] = pred ? 1u : 0u;
    emu::yield_collective();
    const unsigned base = threadIdx.x & ~63u;
    unsigned long long m = 0;
    for (unsigned l = 0; l < 64; ++l)
        if (base + l < blockDim.x && !emu::lane_done(base + l) && emu::slots(p)[base + l]) m |= 1ull << l;
    return m;
}

inline void __syncthreads() { emu::syncthreads(); }

// every lane of the wave reaches the barrier before any lane goes on
inline void emu_wave_barrier() { (void)__ballot(1); }
#define __builtin_amdgcn_wave_barrier() emu_wave_barrier()
#define __builtin_amdgcn_fence(order, scope) std::atomic_thread_fence(std::memory_order_seq_cst)

// ---------------------------------------------------------------- atomics
inline uint32_t atomicAdd(uint32_t* p, uint32_t v) { return std::atomic_ref<uint32_t>(*p).fetch_add(v); }
inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v)
{
    return std::atomic_ref<unsigned long long>(*p).fetch_add(v);
}
inline unsigned long long atomicOr(unsigned long long* p, unsigned long long v)
{
    return std::atomic_ref<unsigned long long>(*p).fetch_or(v);
}
inline float unsafeAtomicAdd(float* p, float v) { return std::atomic_ref<float>(*p).fetch_add(v); }
inline float atomicAdd(float* p, float v) { return std::atomic_ref<float>(*p).fetch_add(v); }
inline double atomicAdd(double* p, double v) { return std::atomic_ref<double>(*p).fetch_add(v); }

// ---------------------------------------------------------------- buffer resources
struct emu_rsrc { const char* p; uint32_t bytes; };
#define __amdgpu_buffer_rsrc_t emu_rsrc
inline emu_rsrc emu_make_rsrc(void* p, short, int bytes, int) { return {(const char*)p, (uint32_t)bytes}; }
#define __builtin_amdgcn_make_buffer_rsrc(p, s, n, f) emu_make_rsrc(p, s, n, f)
inline uint32_t emu_raw_load_b32(emu_rsrc r, uint32_t off, int, int)
{
    if ((uint64_t)off + 4 > r.bytes) return 0u;
    uint32_t v;
    memcpy(&v, r.p + off, 4);
    return v;
}
#define __builtin_amdgcn_raw_buffer_load_b32(r, o, s, a) emu_raw_load_b32(r, o, s, a)
struct emu_u32x4 { uint32_t v[4]; };
inline emu_u32x4 emu_raw_load_b128(emu_rsrc r, uint32_t off, int, int)
{
    emu_u32x4 x{};
    if ((uint64_t)off + 16 > r.bytes) return x;
    memcpy(x.v, r.p + off, 16);
    return x;
}
#define __builtin_amdgcn_raw_buffer_load_b128(r, o, s, a) emu_raw_load_b128(r, o, s, a)

// hardware reciprocal (v_rcp_f32, within 1 ulp).  The library uses it in two ways: the
// culling's corner projections, which allow one ulp and a pixel of slack, and recip(),
// whose one Newton step makes it the IEEE quotient (checked on the hardware over all 2^32
// inputs; a one-ulp-off model breaks that for some inputs, which the hardware's does not).
// The emulation returns the correctly rounded quotient.
inline float emu_rcpf(float x) { return 1.0f / x; }
#define __builtin_amdgcn_rcpf(x) emu_rcpf(x)

// v_mul_u32_u24: the low 32 bits of the product of the operands' low 24 bits.
inline unsigned __umul24(unsigned a, unsigned b) { return (a & 0xFFFFFFu) * (b & 0xFFFFFFu); }

// ---------------------------------------------------------------- runtime API
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorInvalidDevice = 101, hipErrorNotSupported = 801 };
typedef struct emu_stream* hipStream_t;
typedef struct emu_event* hipEvent_t;
typedef struct emu_graph* hipGraph_t;
typedef struct emu_graph_exec* hipGraphExec_t;
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 1 };
enum { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipHostMallocDefault = 0 };
enum hipStreamCaptureMode { hipStreamCaptureModeThreadLocal = 1 };

hipError_t hipGetDevice(int* d);
hipError_t hipSetDevice(int d);
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int d);
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void* f, int block, size_t sh);
template <class F>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, F f, int block, size_t sh)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, (const void*)f, block, sh);
}
hipError_t hipMallocAsync(void** p, size_t n, hipStream_t s);
hipError_t hipFreeAsync(void* p, hipStream_t s);
hipError_t hipMalloc(void** p, size_t n);
template <class T>
inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc((void**)p, n); }
hipError_t hipFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t n, int k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, int k, hipStream_t st);
hipError_t hipHostMalloc(void** p, size_t n, int f);
hipError_t hipHostFree(void* p);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, int f);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, int f);
typedef struct emu_pool* hipMemPool_t;
enum hipMemPoolAttr { hipMemPoolAttrReleaseThreshold = 4 };
inline hipError_t hipDeviceGetDefaultMemPool(hipMemPool_t* p, int) { *p = nullptr; return hipSuccess; }
inline hipError_t hipMemPoolSetAttribute(hipMemPool_t, hipMemPoolAttr, void*) { return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, void*, size_t);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGetLastError();
// the emulated device is the host: a device symbol's address is its host address
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = const_cast<void*>(sym); return hipSuccess; }
const char* hipGetErrorString(hipError_t e);

// kernel launch: run the grid now (stream order = program order)
namespace emu {
void run_grid(const void* kernel, dim3 grid, dim3 block, const std::function<void()>& body);
}
template <class K, class... A>
inline void emu_launch(K kernel, dim3 grid, dim3 block, size_t, hipStream_t, A... args)
{
    emu::run_grid((const void*)kernel, grid, block, [=]() { kernel(args...); });
}
#define hipLaunchKernelGGL(k, g, b, sh, st, ...) emu_launch(k, g, b, sh, st, __VA_ARGS__)
