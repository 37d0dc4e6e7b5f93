// Exhaustive check, over all 2^32 words, of the bracket the walk kernel puts around the
// exact holding-time logarithm: |fast(w) - exact(w)| <= kFastLogAbs + kFastLogRel * fast(w).
// Prints the largest ratio |fast - exact| / (kFastLogAbs + kFastLogRel * fast) and the
// word where it occurs; the check passes when the ratio is below one.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "../../paper_1904_12754_amd/csrc/common.h"

namespace mlmc {
void set_error(const std::string &) {}
}

using namespace mlmc;

constexpr unsigned kThreads = 256;
constexpr unsigned kBlocks = 1u << 14;
constexpr unsigned kPerThread = 1u << 10;   // kThreads * kBlocks * kPerThread = 2^32

__global__ void check(double *ratio_out, unsigned *word_out)
{
    const unsigned tid = blockIdx.x * kThreads + threadIdx.x;
    double worst = 0.0;
    unsigned worst_w = 0;
    for (unsigned i = 0; i < kPerThread; ++i) {
        const unsigned w = tid * kPerThread + i;
        const double ex = neg_log_uniform(w);
        const float fa = neg_log_uniform_fast(w);
        const double bound = static_cast<double>(kFastLogAbs) + static_cast<double>(kFastLogRel) * fa;
        const double r = fabs(static_cast<double>(fa) - ex) / bound;
        if (r > worst) {
            worst = r;
            worst_w = w;
        }
    }
    ratio_out[tid] = worst;
    word_out[tid] = worst_w;
}

int main()
{
    const size_t n = static_cast<size_t>(kThreads) * kBlocks;
    double *d_ratio = nullptr;
    unsigned *d_word = nullptr;
    if (hipMalloc(&d_ratio, n * sizeof(double)) != hipSuccess) return 2;
    if (hipMalloc(&d_word, n * sizeof(unsigned)) != hipSuccess) return 2;
    hipLaunchKernelGGL(check, dim3(kBlocks), dim3(kThreads), 0, 0, d_ratio, d_word);
    if (hipDeviceSynchronize() != hipSuccess) return 3;
    double *h_ratio = new double[n];
    unsigned *h_word = new unsigned[n];
    if (hipMemcpy(h_ratio, d_ratio, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return 4;
    if (hipMemcpy(h_word, d_word, n * sizeof(unsigned), hipMemcpyDeviceToHost) != hipSuccess) return 4;
    double worst = 0.0;
    unsigned worst_w = 0;
    for (size_t i = 0; i < n; ++i)
        if (h_ratio[i] > worst) {
            worst = h_ratio[i];
            worst_w = h_word[i];
        }
    std::printf("max_ratio %.6e word %u\n", worst, worst_w);
    delete[] h_ratio;
    delete[] h_word;
    hipFree(d_ratio);
    hipFree(d_word);
    return worst < 1.0 ? 0 : 1;
}
