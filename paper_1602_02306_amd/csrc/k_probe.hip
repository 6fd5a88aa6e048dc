// Bandwidth probes: simple streams that bound what the estimator's sweeps can
// reach on this device, measured with the same HIP events as the library's
// own kernels (a roofline fraction is then quoted against both the data-sheet
// peak and what a tuned stream of the same read/write mix attains).
//   copy : b = a, 16 bytes per lane, four loads in flight per lane, non-temporal
//   read : sum of a, 16 bytes per lane
//   mix  : w <- w - sum_{l<16} c_l q_l over 17 streams of `slot` bytes: the
//          read/write mix of one Gram-Schmidt update sweep (16 basis vectors
//          read, one vector read and written in place)
#include <hip/hip_runtime.h>

#include "ecount.h"
#include "ecount_internal.h"

namespace ecnt {

typedef double pd2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void k_probe_copy(const pd2 *__restrict__ a, pd2 *__restrict__ b, size_t n2)
{
    size_t i = (size_t)blockIdx.x * 1024 + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * 1024;
    for (; i + 768 < n2; i += stride) {
        pd2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(a + i + u * 256);
#pragma unroll
        for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], b + i + u * 256);
    }
}

__global__ __launch_bounds__(256) void k_probe_read(const pd2 *__restrict__ a, size_t n2, double *__restrict__ sink)
{
    size_t i = (size_t)blockIdx.x * 1024 + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * 1024;
    double s = 0.0;
    for (; i + 768 < n2; i += stride) {
        pd2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(a + i + u * 256);
#pragma unroll
        for (int u = 0; u < 4; ++u) s += v[u].x + v[u].y;
    }
    if (s == -1.0) sink[0] = s;   // keeps the loads; never true for the zero-filled probe buffer
}

__global__ __launch_bounds__(256) void k_probe_mix(const pd2 *__restrict__ q, size_t ss2, pd2 *__restrict__ w,
                                                   size_t n2)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * 256;
    for (; i < n2; i += stride) {
        pd2 x = w[i];
        pd2 v[16];
#pragma unroll
        for (int l = 0; l < 16; ++l) v[l] = __builtin_nontemporal_load(q + l * ss2 + i);
#pragma unroll
        for (int l = 0; l < 16; ++l) x -= (0.001 * (l + 1)) * v[l];
        w[i] = x;
    }
}

// Times `reps` launches of probe `kind` on the buffer; returns GB/s (bytes moved / time).
int run_probe(int kind, void *buf, size_t bytes, int reps, hipStream_t st, double *gbs)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1;
    const size_t slot = kind == 2 ? (bytes / 17) / 4096 * 4096 : bytes / 2;
    const size_t n2 = slot / 16;
    pd2 *a = (pd2 *)buf, *b = (pd2 *)((char *)buf + slot);
    double moved = 0.0;
    auto launch = [&]() {
        if (kind == 0) k_probe_copy<<<16384, 256, 0, st>>>(a, b, n2);
        else if (kind == 1) k_probe_read<<<16384, 256, 0, st>>>(a, n2, (double *)b);
        else k_probe_mix<<<8192, 256, 0, st>>>(a, n2, (pd2 *)((char *)buf + 16 * slot), n2);
    };
    if (kind == 0) moved = 2.0 * (double)(n2 / 1024 * 1024) * 16;
    else if (kind == 1) moved = (double)(n2 / 1024 * 1024) * 16;
    else moved = 18.0 * (double)n2 * 16;
    (void)hipMemsetAsync(buf, 0, kind == 2 ? 17 * slot : 2 * slot, st);
    launch();   // warm-up
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r) launch();
    (void)hipEventRecord(e1, st);
    hipError_t e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess || ms <= 0.f) return -1;
    *gbs = moved * reps / (ms / 1e3) / 1e9;
    return 0;
}

}  // namespace ecnt
