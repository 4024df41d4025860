// iblb_probe_phase_sync: what it costs to order two phases of a step across
// the whole GPU, by a kernel boundary or by a grid-wide barrier inside one
// cooperative kernel.  The batched step orders its phases by kernel
// boundaries; this measurement is the reason.
#include "iblb.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

namespace {

constexpr int kProbeThreads = 256;
constexpr long kSpinLimit = 1l << 22;  // sleeps of one wait before it gives up (about 0.1 s)

// One phase of the boundary variant: each block writes one word.
__global__ __launch_bounds__(kProbeThreads) void k_probe_phase(unsigned *words, unsigned r)
{
    if (threadIdx.x == 0)
        words[blockIdx.x] = r;
}

// Grid-wide barrier: sync[0] counts the blocks that arrived, sync[1] is the
// generation.  The block that arrives last resets the count and advances the
// generation; the others wait for the generation to change, at most
// kSpinLimit sleeps, after which the barrier and every later one return at
// once with *timeout set, so that the kernel ends even if its blocks were not
// all resident.
__device__ void grid_barrier(unsigned *sync, unsigned nblocks, int *timeout)
{
    __syncthreads();
    if (threadIdx.x == 0 && __hip_atomic_load(timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        const unsigned g = __hip_atomic_load(&sync[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (__hip_atomic_fetch_add(&sync[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == nblocks - 1) {
            __hip_atomic_store(&sync[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&sync[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long spins = 0;
            while (__hip_atomic_load(&sync[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (++spins > kSpinLimit) {
                    __hip_atomic_store(timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
    }
    __syncthreads();
}

// The barrier variant: `rounds` phases in one kernel, each block writing one
// word per phase and then passing the barrier.
__global__ __launch_bounds__(kProbeThreads) void k_probe_barriers(unsigned *words, unsigned *sync, int rounds,
                                                                  int *timeout)
{
    for (int r = 0; r < rounds; ++r) {
        if (threadIdx.x == 0)
            words[blockIdx.x] = (unsigned)r;
        grid_barrier(sync, gridDim.x, timeout);
    }
}

struct Probe {
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *buf = nullptr;
    ~Probe()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (buf) (void)hipFree(buf);
        if (s) (void)hipStreamDestroy(s);
    }
};

double median(std::vector<double> v)
{
    std::sort(v.begin(), v.end());
    return v[v.size() / 2];
}

}  // namespace

#define PROBE_TRY(expr)                          \
    do {                                         \
        if ((expr) != hipSuccess) return IBLB_E_DEVICE; \
    } while (0)

int iblb_probe_phase_sync(int32_t blocks, int32_t rounds, double *boundary_us, double *barrier_us)
{
    if (blocks < 1 || rounds < 1 || rounds > 100000 || !boundary_us || !barrier_us) return IBLB_E_INVAL;
    int dev = 0, cus = 0, per_cu = 0, coop = 0;
    PROBE_TRY(hipGetDevice(&dev));
    PROBE_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    PROBE_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    PROBE_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_probe_barriers, kProbeThreads, 0));
    if (!coop || blocks > per_cu * cus) return IBLB_E_INVAL;  // the barrier needs every block resident
    Probe P;
    PROBE_TRY(hipStreamCreateWithFlags(&P.s, hipStreamNonBlocking));
    PROBE_TRY(hipEventCreate(&P.e0));
    PROBE_TRY(hipEventCreate(&P.e1));
    // words [blocks], then sync [2] and the timeout flag
    PROBE_TRY(hipMalloc(&P.buf, (size_t)blocks * 4 + 256));
    unsigned *words = (unsigned *)P.buf;
    unsigned *sync = (unsigned *)((char *)P.buf + ((size_t)blocks * 4 + 127) / 128 * 128);
    int *timeout = (int *)(sync + 2);
    // kernel boundaries: `rounds` launches captured in one graph
    PROBE_TRY(hipStreamBeginCapture(P.s, hipStreamCaptureModeThreadLocal));
    for (int r = 0; r < rounds; ++r) k_probe_phase<<<blocks, kProbeThreads, 0, P.s>>>(words, (unsigned)r);
    PROBE_TRY(hipStreamEndCapture(P.s, &P.graph));
    PROBE_TRY(hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0));
    PROBE_TRY(hipGraphLaunch(P.exec, P.s));  // warm-up
    std::vector<double> tb, tg;
    for (int rep = 0; rep < 5; ++rep) {
        float ms = 0.f;
        PROBE_TRY(hipEventRecord(P.e0, P.s));
        PROBE_TRY(hipGraphLaunch(P.exec, P.s));
        PROBE_TRY(hipEventRecord(P.e1, P.s));
        PROBE_TRY(hipEventSynchronize(P.e1));
        PROBE_TRY(hipEventElapsedTime(&ms, P.e0, P.e1));
        tb.push_back(1e3 * ms / rounds);
    }
    // grid barriers: one cooperative kernel per repetition
    for (int rep = 0; rep < 6; ++rep) {
        PROBE_TRY(hipMemsetAsync(sync, 0, 16, P.s));
        int r = rounds;
        void *args[] = {&words, &sync, &r, &timeout};
        float ms = 0.f;
        PROBE_TRY(hipEventRecord(P.e0, P.s));
        PROBE_TRY(hipLaunchCooperativeKernel((const void *)k_probe_barriers, dim3(blocks), dim3(kProbeThreads), args,
                                             0, P.s));
        PROBE_TRY(hipEventRecord(P.e1, P.s));
        PROBE_TRY(hipEventSynchronize(P.e1));
        PROBE_TRY(hipEventElapsedTime(&ms, P.e0, P.e1));
        unsigned st[3] = {0, 0, 0};
        PROBE_TRY(hipMemcpy(st, sync, 12, hipMemcpyDeviceToHost));
        if (st[2] != 0 || st[1] != (unsigned)rounds) return IBLB_E_UNSTABLE;  // a wait gave up
        if (rep > 0) tg.push_back(1e3 * ms / rounds);  // the first launch warms up
    }
    *boundary_us = median(tb);
    *barrier_us = median(tg);
    return IBLB_OK;
}
