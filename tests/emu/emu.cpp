// CPU emulation build of libkfvol: the library's own sources compiled for the host
// against emu_shim.h, with a fiber scheduler standing in for waves and blocks.
#include "emu_shim.h"

#include <mutex>
#include <thread>

// Minimal x86-64 System V context switch: saves the callee-saved registers, MXCSR and the
// x87 control word on the current stack, stores the stack pointer in *save_sp and resumes
// the context whose stack pointer is new_sp.
extern "C" void emu_ctx_switch(void** save_sp, void* new_sp);
asm(R"(
.text
.globl emu_ctx_switch
.type emu_ctx_switch,@function
emu_ctx_switch:
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
.size emu_ctx_switch, .-emu_ctx_switch
)");

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#include <sanitizer/asan_interface.h>
#include <sanitizer/common_interface_defs.h>
#define EMU_ASAN 1
#endif
#endif

thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;

#include "kf_integrate.hip"
#include "kf_backward.hip"
#include "kf_raycast.hip"
#include "kf_texture.hip"
#include "kf_mesh.hip"
#include "kf_capi.hip"
#include "kf_decimate.cpp"

namespace emu {

constexpr size_t kStack = 64 * 1024;

struct Fiber {
    void* sp = nullptr;
    char* stack = nullptr;
    bool done = false;
};

struct Block {
    void* sched_sp = nullptr;
    std::vector<Fiber> f;
    std::vector<uint64_t> slot[2];
    std::vector<int> par;
    int cur = -1;
    int alive = 0;
    int bar_arrived = 0;
    unsigned bar_gen = 0;
    const std::function<void()>* body = nullptr;
    const void* sched_bottom = nullptr;
    size_t sched_size = 0;
};

thread_local Block* g_blk = nullptr;
thread_local bool g_direct = false;

void check_direct(const char* what)
{
    if (g_direct) {
        fprintf(stderr, "emu: %s in a kernel run without fibers\n", what);
        abort();
    }
}

uint64_t* slots(int p) { return g_blk->slot[p].data(); }
int next_parity()
{
    int& p = g_blk->par[threadIdx.x];
    const int r = p;
    p ^= 1;
    return r;
}
bool lane_done(unsigned tid) { return g_blk->f[tid].done; }

static void to_scheduler(bool finishing)
{
    Block* B = g_blk;
    Fiber& me = B->f[B->cur];
#ifdef EMU_ASAN
    void* fake = nullptr;
    __sanitizer_start_switch_fiber(finishing ? nullptr : &fake, B->sched_bottom, B->sched_size);
#endif
    emu_ctx_switch(&me.sp, B->sched_sp);
#ifdef EMU_ASAN
    __sanitizer_finish_switch_fiber(fake, &B->sched_bottom, &B->sched_size);
#endif
    (void)finishing;
}

void yield_collective() { to_scheduler(false); }

void syncthreads()
{
    if (g_direct) check_direct("__syncthreads");
    Block* B = g_blk;
    const unsigned gen = B->bar_gen;
    ++B->bar_arrived;
    while (B->bar_gen == gen) to_scheduler(false);
}

[[noreturn]] static void fiber_entry()
{
    Block* B = g_blk;
#ifdef EMU_ASAN
    __sanitizer_finish_switch_fiber(nullptr, &B->sched_bottom, &B->sched_size);
#endif
    (*B->body)();
    B->f[B->cur].done = true;
    --B->alive;
    to_scheduler(true);
    abort();   // a finished fiber is never resumed
}

// Initial stack of a fiber, laid out as emu_ctx_switch expects to find it: control words,
// six callee-saved registers, then the entry address as the return address (and a zero
// slot so that the entry sees the stack alignment of a called function).
static void* fiber_stack_init(char* stack, size_t size)
{
    uintptr_t top = ((uintptr_t)(stack + size)) & ~(uintptr_t)15;
    uint64_t* sp = (uint64_t*)top;
    *--sp = 0;                              // alignment slot / fake return address
    *--sp = (uint64_t)(uintptr_t)&fiber_entry;
    for (int r = 0; r < 6; ++r) *--sp = 0;  // rbp rbx r12 r13 r14 r15
    *--sp = 0x037F00001F80ull;              // MXCSR 0x1F80 | x87 control word 0x037F << 32
    return sp;
}

static void run_block_fibers(Block& B, unsigned n, const std::function<void()>& body)
{
    if (B.f.size() < n) {
        B.f.resize(n);
        for (auto& fb : B.f)
            if (!fb.stack) fb.stack = (char*)malloc(kStack);
    }
    for (int p = 0; p < 2; ++p) B.slot[p].assign(n, 0);
    B.par.assign(n, 0);
    B.body = &body;
    B.alive = (int)n;
    B.bar_arrived = 0;
    for (unsigned t = 0; t < n; ++t) {
        Fiber& fb = B.f[t];
        fb.done = false;
#ifdef EMU_ASAN
        // a finished fiber never unwinds its frames: clear their redzones before reuse
        __asan_unpoison_memory_region(fb.stack, kStack);
#endif
        fb.sp = fiber_stack_init(fb.stack, kStack);
    }
    g_blk = &B;
    while (B.alive > 0) {
        for (unsigned t = 0; t < n; ++t) {
            if (B.f[t].done) continue;
            B.cur = (int)t;
            threadIdx = dim3(t, 0, 0);
#ifdef EMU_ASAN
            void* fake = nullptr;
            __sanitizer_start_switch_fiber(&fake, B.f[t].stack, kStack);
#endif
            emu_ctx_switch(&B.sched_sp, B.f[t].sp);
#ifdef EMU_ASAN
            __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#endif
        }
        if (B.bar_arrived > 0 && B.bar_arrived == B.alive) {
            B.bar_arrived = 0;
            ++B.bar_gen;
        }
    }
    g_blk = nullptr;
}

template <int MODE, int KIND, int... SH>
static bool is_integrate(const void* k, std::integer_sequence<int, SH...>)
{
    return ((k == (const void*)kf::integrate_kernel<MODE, KIND, SH>) || ...);
}

static bool needs_fibers(const void* k)
{
    using Seq = std::make_integer_sequence<int, kf::N_BRICK_SHAPES>;
    if (is_integrate<kf::MODE_INTEGRATE, kf::KIND_GEOM>(k, Seq{}) ||
        is_integrate<kf::MODE_INTEGRATE, kf::KIND_COLOUR>(k, Seq{}) ||
        is_integrate<kf::MODE_COUNT, kf::KIND_GEOM>(k, Seq{}) ||
        is_integrate<kf::MODE_COUNT, kf::KIND_COLOUR>(k, Seq{}))
        return true;
    static const void* list[] = {
        (const void*)kf::pyramid_up_kernel,
        (const void*)kf::status_kernel<true>,
        (const void*)kf::status_kernel<false>,
        (const void*)kf::cull_kernel,
        (const void*)kf::backward_cull_kernel,
        (const void*)kf::reduce_xi_kernel,
        (const void*)kf::texture_kernel,
        (const void*)kf::mc_classify_kernel,
        (const void*)kf::mc_block_sums_kernel,
        (const void*)kf::mc_scan_blocks_kernel,
        (const void*)kf::mc_vertices_kernel,
        (const void*)kf::mc_triangles_kernel,
        (const void*)kf::backward_kernel<32, false>,
        (const void*)kf::backward_kernel<64, false>,
        (const void*)kf::backward_kernel<32, true>,
        (const void*)kf::backward_kernel<64, true>,
        (const void*)kf::bin_scan_kernel,
        (const void*)kf::backward_image_kernel,
    };
    for (const void* p : list)
        if (p == k) return true;
    return false;
}

int n_workers()
{
    const char* v = getenv("EMU_THREADS");
    return v ? atoi(v) : 8;
}

void run_grid(const void* kernel, dim3 grid, dim3 block, const std::function<void()>& body)
{
    const bool fibers = needs_fibers(kernel);
    const unsigned nb = grid.x * grid.y * grid.z;
    const unsigned nt = block.x * block.y * block.z;
    std::atomic<unsigned> next{0};
    auto worker = [&]() {
        Block B;
        for (;;) {
            const unsigned b = next.fetch_add(1);
            if (b >= nb) break;
            blockIdx = dim3(b % grid.x, (b / grid.x) % grid.y, b / (grid.x * grid.y));
            blockDim = block;
            gridDim = grid;
            if (fibers) {
                run_block_fibers(B, nt, body);
            } else {
                g_direct = true;
                for (unsigned t = 0; t < nt; ++t) {
                    threadIdx = dim3(t, 0, 0);
                    body();
                }
                g_direct = false;
            }
        }
        for (auto& fb : B.f) free(fb.stack);
    };
    const int nw = std::max(1, std::min<int>(n_workers(), (int)nb));
    std::vector<std::thread> th;
    for (int w = 1; w < nw; ++w) th.emplace_back(worker);
    worker();
    for (auto& t : th) t.join();
}

}  // namespace emu

// ---------------------------------------------------------------- runtime API
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 8; return hipSuccess; }
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void*, int, size_t) { *n = 1; return hipSuccess; }
hipError_t hipMallocAsync(void** p, size_t n, hipStream_t) { *p = malloc(n ? n : 1); return *p ? hipSuccess : 2; }
hipError_t hipFreeAsync(void* p, hipStream_t) { free(p); return hipSuccess; }
hipError_t hipMalloc(void** p, size_t n) { *p = malloc(n ? n : 1); return *p ? hipSuccess : 2; }
hipError_t hipFree(void* p) { free(p); return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, int) { memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, int, hipStream_t) { memcpy(d, s, n); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t n, int) { *p = malloc(n ? n : 1); return hipSuccess; }
hipError_t hipHostFree(void* p) { free(p); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, int) { *e = (hipEvent_t)malloc(8); return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, int) { *s = (hipStream_t)malloc(8); return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = nullptr; return hipErrorNotSupported; }
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, void*, void*, size_t) { return hipErrorNotSupported; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "emulated HIP error"; }
