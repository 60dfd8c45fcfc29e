// Measurement probe (not part of libdemons): the cost of a grid-wide barrier
// (cooperative groups) on this device, the step a persistent kernel would
// need between the pre-warp, force and smoothing of every iteration.  Each
// block writes its own words, then the grid synchronises; the time per
// barrier is reported for 1 to 8 co-resident blocks per compute unit.
// Output: one JSON object per configuration on stdout.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>
#include <stdio.h>

namespace cg = cooperative_groups;

__global__ void k_barriers(int iters, float *buf, int words_per_block)
{
    cg::grid_group g = cg::this_grid();
    for (int i = 0; i < iters; ++i) {
        for (int w = threadIdx.x; w < words_per_block; w += blockDim.x)
            buf[(size_t)blockIdx.x * words_per_block + w] = (float)i;
        g.sync();
    }
}

#define CHECK(x)                                                                  \
    do {                                                                          \
        hipError_t e_ = (x);                                                      \
        if (e_ != hipSuccess) {                                                   \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));               \
            return 1;                                                             \
        }                                                                         \
    } while (0)

int main()
{
    int ncu = 0, per_cu = 0;
    CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0));
    CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_barriers, 256, 0));
    const int max_words = 8192;
    float *buf = nullptr;
    CHECK(hipMalloc(&buf, sizeof(float) * (size_t)ncu * (per_cu > 8 ? 8 : per_cu) * max_words));
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    for (int bpc = 1; bpc <= 8 && bpc <= per_cu; bpc *= 2) {
        for (int words : {0, 1024, max_words}) {
            int iters = 200, blocks = ncu * bpc;
            void *args[] = {&iters, &buf, &words};
            CHECK(hipLaunchCooperativeKernel((void *)k_barriers, dim3(blocks), dim3(256), args, 0, 0));  // warm-up
            CHECK(hipDeviceSynchronize());
            CHECK(hipEventRecord(a, 0));
            CHECK(hipLaunchCooperativeKernel((void *)k_barriers, dim3(blocks), dim3(256), args, 0, 0));
            CHECK(hipEventRecord(b, 0));
            CHECK(hipEventSynchronize(b));
            float ms = 0.0f;
            CHECK(hipEventElapsedTime(&ms, a, b));
            printf("{\"blocks\": %d, \"blocks_per_cu\": %d, \"words_per_block\": %d, \"us_per_barrier\": %.2f}\n",
                   blocks, bpc, words, ms * 1e3 / iters);
            fflush(stdout);
        }
    }
    CHECK(hipFree(buf));
    return 0;
}
