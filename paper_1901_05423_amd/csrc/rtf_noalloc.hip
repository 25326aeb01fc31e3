// rtf_noalloc.hip -- rtf_backward_static: the backward pass with its scratch
// (the per-element sums B and D, the per-distribution sums A, the combining
// pass's chunk heads, links and carries) in a fixed device array of this file
// instead of a caller workspace, for callers that cannot allocate device
// memory.  The kernels are those of rtf_backward.
#include <mutex>

#include "rtf_internal.h"

using namespace rtf;

namespace {

constexpr int64_t STATIC_MAX_N = RTF_BACKWARD_STATIC_MAX_N;
constexpr int32_t STATIC_MAX_D = RTF_BACKWARD_STATIC_MAX_D;
constexpr size_t STATIC_BYTES = backward_layout(STATIC_MAX_D, STATIC_MAX_N, nullptr, nullptr);

// One copy per GPU, held until the process ends.  Host code never uses this
// name as an address: it reaches the array through the per-device pointer
// hipGetSymbolAddress returns.
static __device__ __align__(256) char scratch[STATIC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
char *g_ptr[MAX_DEVICES] = {};

// The device address of the current device's copy of `scratch`, looked up
// once per device with that device current.
rtf_status scratch_ptr(char **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return RTF_ERR_HIP;
    if (dev < 0 || dev >= MAX_DEVICES) return RTF_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RTF_ERR_HIP;
        g_ptr[dev] = static_cast<char *>(p);
    }
    *out = g_ptr[dev];
    return RTF_OK;
}

}  // namespace

rtf_status rtf_backward_static(const rtf_forest *f, const int64_t *sample_off, const uint64_t *u,
                               const int32_t *idx, const double *grad_x, int64_t S,
                               const double *scale, double *grad_w, hipStream_t stream) {
    if (!f) return RTF_ERR_INVALID_ARG;
    if (f->n_total > STATIC_MAX_N || f->D > STATIC_MAX_D) return RTF_ERR_SIZE;
    char *base = nullptr;
    const rtf_status st = scratch_ptr(&base);
    if (st != RTF_OK) return st;
    BackwardScratch w;
    backward_layout(f->D, f->n_total, base, &w);
    return backward_enqueue(f, sample_off, u, idx, grad_x, S, scale, grad_w, w, stream);
}
