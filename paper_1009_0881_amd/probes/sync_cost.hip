// Cost of one grid-wide barrier inside a kernel against one kernel boundary
// on a stream: the measurement behind running each sweep iteration as a few
// dependent launches instead of one persistent kernel.
//
//   sync_cost [blocks ...]        (default: 64 128 256 512)
//
// For each grid size (256 threads per block) it prints one JSON line:
//   boundary_us  events around K back-to-back launches of an empty kernel of
//                that grid on one stream, divided by K;
//   barrier_us   (T(R) - T(0)) / R, where T(R) is the event time of one
//                cooperative launch whose blocks meet at R grid-wide barriers
//                (device-scope atomic counter, release on arrival, acquire
//                while waiting), median of several launches.
// Every wait is bounded: a block that polls past the cap sets a failure flag
// and goes on, so every launch ends; a run with the flag set is reported as
// failed.  Grids that cannot all be resident at once are skipped (the
// cooperative launch would be rejected).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                       \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));               \
            std::exit(1);                                                              \
        }                                                                              \
    } while (0)

namespace {

constexpr int kThreads = 256;
constexpr int kBoundaryLaunches = 2000;
constexpr int kRounds = 200;
constexpr int kPollCap = 20000;   // about 20 ms of polling per barrier at most
constexpr int kReps = 7;

__global__ __launch_bounds__(kThreads) void k_empty(unsigned *sink) {
    // never taken; keeps the launch from being optimised into nothing
    if (sink != nullptr && blockIdx.x == 0x7fffffffu) sink[threadIdx.x] = 1u;
}

__global__ __launch_bounds__(kThreads) void k_rounds(unsigned *ctr, unsigned *fail, int rounds) {
    const unsigned nb = gridDim.x;
    for (int i = 1; i <= rounds; ++i) {
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned target = nb * (unsigned)i;
            int polls = 0;
            while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (++polls > kPollCap) {
                    __hip_atomic_fetch_or(fail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
    }
}

float elapsed_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    CHECK(hipEventElapsedTime(&ms, a, b));
    return ms;
}

// median event time (ms) of one cooperative launch with the given rounds
float time_rounds(int blocks, int rounds, unsigned *ctr, unsigned *fail, hipStream_t s,
                  hipEvent_t e0, hipEvent_t e1, bool &failed) {
    std::vector<float> t;
    for (int rep = 0; rep < kReps + 1; ++rep) {
        CHECK(hipMemsetAsync(ctr, 0, sizeof(unsigned), s));
        void *args[] = {&ctr, &fail, &rounds};
        CHECK(hipEventRecord(e0, s));
        CHECK(hipLaunchCooperativeKernel((const void *)k_rounds, dim3(blocks), dim3(kThreads), args,
                                         0, s));
        CHECK(hipEventRecord(e1, s));
        CHECK(hipStreamSynchronize(s));
        if (rep > 0) t.push_back(elapsed_ms(e0, e1));   // the first launch warms up
    }
    unsigned f = 0;
    CHECK(hipMemcpy(&f, fail, sizeof(unsigned), hipMemcpyDeviceToHost));
    failed = failed || f != 0;
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

}  // namespace

int main(int argc, char **argv) {
    std::vector<int> grids;
    for (int i = 1; i < argc; ++i) grids.push_back(std::atoi(argv[i]));
    if (grids.empty()) grids = {64, 128, 256, 512};

    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    CHECK(hipGetDevice(&dev));
    CHECK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_rounds, kThreads, 0));
    if (!coop) {
        std::fprintf(stderr, "device does not support cooperative launches\n");
        return 1;
    }
    hipStream_t s;
    CHECK(hipStreamCreate(&s));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    unsigned *buf = nullptr;
    CHECK(hipMalloc(&buf, 2 * sizeof(unsigned)));
    CHECK(hipMemset(buf, 0, 2 * sizeof(unsigned)));
    unsigned *ctr = buf, *fail = buf + 1;

    for (int blocks : grids) {
        if (blocks < 1 || blocks > per_cu * cus) {
            std::printf("{\"blocks\": %d, \"skipped\": \"more blocks than can be resident (%d)\"}\n",
                        blocks, per_cu * cus);
            continue;
        }
        // kernel boundary: back-to-back empty launches on one stream
        for (int i = 0; i < 50; ++i) k_empty<<<blocks, kThreads, 0, s>>>(nullptr);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e0, s));
        for (int i = 0; i < kBoundaryLaunches; ++i) k_empty<<<blocks, kThreads, 0, s>>>(nullptr);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e1, s));
        CHECK(hipStreamSynchronize(s));
        const double boundary_us = 1e3 * elapsed_ms(e0, e1) / kBoundaryLaunches;

        bool failed = false;
        const float t0 = time_rounds(blocks, 0, ctr, fail, s, e0, e1, failed);
        const float tr = time_rounds(blocks, kRounds, ctr, fail, s, e0, e1, failed);
        const double barrier_us = 1e3 * (tr - t0) / kRounds;
        std::printf("{\"blocks\": %d, \"threads_per_block\": %d, \"boundary_us\": %.3f, "
                    "\"barrier_us\": %.3f, \"rounds\": %d, \"launch_0_rounds_us\": %.3f, "
                    "\"launch_%d_rounds_us\": %.3f, \"failed\": %s}\n",
                    blocks, kThreads, boundary_us, barrier_us, kRounds, 1e3 * t0, kRounds, 1e3 * tr,
                    failed ? "true" : "false");
        std::fflush(stdout);
    }
    CHECK(hipFree(buf));
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    CHECK(hipStreamDestroy(s));
    return 0;
}
