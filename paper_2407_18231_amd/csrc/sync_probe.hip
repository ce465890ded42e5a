// sync_probe.hip -- what a stage boundary of the chain costs on this GPU,
// for the choice between one launch per stage and one persistent kernel
// with device-wide barriers between stages.
//
// The same grid (every block co-resident, 256 threads, one element touched
// per thread) crosses `iters` stage boundaries four ways:
//   persistent: one cooperative launch, a cooperative-groups grid barrier
//               after each stage;
//   persistent, own barrier: the same with an atomic counter barrier;
//   graph:      one kernel per stage, replayed from a captured hipGraph;
//   eager:      one kernel per stage, launched one after another.
// Prints one JSON line with the microseconds per boundary of each.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace cg = cooperative_groups;

__global__ __launch_bounds__(256) void k_stage(unsigned *p, unsigned n)
{
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] += 1u;
}

__global__ __launch_bounds__(256) void k_persistent(unsigned *p, unsigned n, unsigned iters)
{
    cg::grid_group grid = cg::this_grid();
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    for (unsigned k = 0; k < iters; k++) {
        if (i < n) p[i] += 1u;
        grid.sync();
    }
}

// The same with a barrier of our own: every block adds one to a counter
// and waits (with a sleep between polls) until the counter reaches the
// number of blocks times the stages passed.  The wait is bounded: after
// kMaxPolls polls a block records a timeout, and once one is recorded no
// block waits any more, so every wave ends.
constexpr unsigned kMaxPolls = 1u << 18;

__global__ __launch_bounds__(256) void k_persistent_own(unsigned *p, unsigned n, unsigned iters, unsigned *bar,
                                                        unsigned *timed_out)
{
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    for (unsigned k = 0; k < iters; k++) {
        if (i < n) p[i] += 1u;
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            atomicAdd(bar, 1u);
            const unsigned target = (k + 1u) * gridDim.x;
            unsigned polls = 0;
            while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                if (++polls == kMaxPolls) atomicOr(timed_out, 1u);
                if (__hip_atomic_load(timed_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
            }
        }
        __syncthreads();
    }
}

#define CHECK(x)                                                                          \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) {                                                           \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                  \
            return 1;                                                                     \
        }                                                                                 \
    } while (0)

int main(int argc, char **argv)
{
    const unsigned iters = argc > 1 ? (unsigned)std::atoi(argv[1]) : 200u;
    int dev = 0, cus = 0, per_cu = 0, coop = 0;
    CHECK(hipSetDevice(dev));
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    CHECK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    int per_cu_own = 0;
    CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent, 256, 0));
    CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_own, k_persistent_own, 256, 0));
    if (per_cu_own < per_cu) per_cu = per_cu_own;     // every block of both kernels co-resident
    if (!coop || per_cu < 1) {
        std::printf("{\"cooperative_launch\": false}\n");
        return 0;
    }
    // the chain's walks take up to 2048 blocks of 256 threads
    unsigned blocks = (unsigned)(cus * per_cu);
    if (blocks > 2048u) blocks = 2048u;
    const unsigned n = blocks * 256u;
    unsigned *p = nullptr;
    CHECK(hipMalloc(&p, sizeof(unsigned) * n));
    CHECK(hipMemset(p, 0, sizeof(unsigned) * n));
    hipStream_t s;
    CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    float ms_p = 0.f, ms_g = 0.f, ms_e = 0.f;
    // persistent kernel with grid barriers (warm-up, then timed)
    unsigned it = iters;
    void *args[] = {&p, (void *)&n, &it};
    for (int rep = 0; rep < 2; rep++) {
        CHECK(hipEventRecord(e0, s));
        CHECK(hipLaunchCooperativeKernel((void *)k_persistent, dim3(blocks), dim3(256), args, 0, s));
        CHECK(hipEventRecord(e1, s));
        CHECK(hipEventSynchronize(e1));
        CHECK(hipEventElapsedTime(&ms_p, e0, e1));
    }
    // persistent kernel with the barrier of our own
    unsigned *bar = nullptr;
    CHECK(hipMalloc(&bar, 2 * sizeof(unsigned)));
    float ms_o = 0.f;
    unsigned timed_out = 0;
    for (int rep = 0; rep < 2; rep++) {
        CHECK(hipMemsetAsync(bar, 0, 2 * sizeof(unsigned), s));
        unsigned *tflag = bar + 1;
        void *oargs[] = {&p, (void *)&n, &it, &bar, &tflag};
        CHECK(hipEventRecord(e0, s));
        CHECK(hipLaunchCooperativeKernel((void *)k_persistent_own, dim3(blocks), dim3(256), oargs, 0, s));
        CHECK(hipEventRecord(e1, s));
        CHECK(hipEventSynchronize(e1));
        CHECK(hipEventElapsedTime(&ms_o, e0, e1));
        CHECK(hipMemcpy(&timed_out, tflag, sizeof(unsigned), hipMemcpyDeviceToHost));
    }
    // one kernel per stage, captured once and replayed
    hipGraph_t graph;
    hipGraphExec_t exec;
    CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (unsigned k = 0; k < iters; k++) k_stage<<<blocks, 256, 0, s>>>(p, n);
    CHECK(hipStreamEndCapture(s, &graph));
    CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    for (int rep = 0; rep < 2; rep++) {
        CHECK(hipEventRecord(e0, s));
        CHECK(hipGraphLaunch(exec, s));
        CHECK(hipEventRecord(e1, s));
        CHECK(hipEventSynchronize(e1));
        CHECK(hipEventElapsedTime(&ms_g, e0, e1));
    }
    // one kernel per stage, launched eagerly
    for (int rep = 0; rep < 2; rep++) {
        CHECK(hipEventRecord(e0, s));
        for (unsigned k = 0; k < iters; k++) k_stage<<<blocks, 256, 0, s>>>(p, n);
        CHECK(hipEventRecord(e1, s));
        CHECK(hipEventSynchronize(e1));
        CHECK(hipEventElapsedTime(&ms_e, e0, e1));
    }
    CHECK(hipGetLastError());
    std::printf("{\"cooperative_launch\": true, \"blocks\": %u, \"threads_per_block\": 256, \"boundaries\": %u, "
                "\"us_per_boundary\": {\"persistent_grid_barrier\": %.3f, \"persistent_own_barrier\": %.3f, "
                "\"graph_launch\": %.3f, \"eager_launch\": %.3f}, \"own_barrier_timed_out\": %s}\n",
                blocks, iters, 1e3 * ms_p / iters, 1e3 * ms_o / iters, 1e3 * ms_g / iters, 1e3 * ms_e / iters,
                timed_out ? "true" : "false");
    (void)hipFree(bar);
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    (void)hipFree(p);
    return 0;
}
