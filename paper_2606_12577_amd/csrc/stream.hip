// Streaming-bandwidth reference for the roofline figures: what plain kernels
// that only stream arrays through HBM reach on this device.  A launch reads
// n_read arrays and writes n_write (0 or 1) of the same length, one 16-byte
// element per thread and a workgroup per 256 elements (the launch shape that
// streams fastest here: persistent grids that loop over the arrays wrote at
// about two thirds of its rate).
#include "cs_internal.h"

namespace cs {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

template <int NR, int NW>
__global__ __launch_bounds__(256) void k_stream(int64_t n, const f4v *__restrict__ a0, const f4v *__restrict__ a1,
                                                const f4v *__restrict__ a2, const f4v *__restrict__ a3,
                                                f4v *__restrict__ w, float *__restrict__ sink) {
    const int64_t i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= n) return;
    f4v s = {1.0f, 2.0f, 3.0f, 4.0f};
    if constexpr (NR > 0) s += a0[i];
    if constexpr (NR > 1) s += a1[i];
    if constexpr (NR > 2) s += a2[i];
    if constexpr (NR > 3) s += a3[i];
    if constexpr (NW > 0) {
        w[i] = s;
    } else if (s.x + s.y + s.z + s.w == -1.0f) {   // never true for the filled inputs: the reads stay
        sink[0] = s.x;
    }
}

__global__ __launch_bounds__(256) void k_stream_fill(int64_t n, f4v *__restrict__ a) {
    const int64_t i = blockIdx.x * 256LL + threadIdx.x;
    if (i < n) a[i] = f4v{0.25f, 0.5f, 0.75f, 1.0f};
}

}  // namespace

void stream_bandwidth(Ctx &c, int n_read, int n_write, int64_t bytes, int reps, double *gbps, double *us) {
    if (n_read < 0 || n_read > 4 || n_write < 0 || n_write > 1 || n_read + n_write == 0)
        fail(CS_EINVAL, "stream probe: n_read must be in [0, 4], n_write in [0, 1], not both 0");
    if (bytes < 16 || bytes % 16 != 0) fail(CS_EINVAL, "stream probe: bytes must be a positive multiple of 16");
    if (bytes > (int64_t(1) << 36)) fail(CS_EINVAL, "stream probe: at most 64 GiB per array");
    if (reps < 1) fail(CS_EINVAL, "stream probe: reps must be at least 1");
    const int64_t n = bytes / 16;
    const int na = n_read + n_write;
    DBuf<f4v> arr[5];
    for (int k = 0; k < na; ++k) arr[k].alloc((size_t)n);
    DBuf<float> sink(1);
    const unsigned G = (unsigned)((n + 255) / 256);
    for (int k = 0; k < na; ++k)
        hipLaunchKernelGGL(k_stream_fill, dim3(G), dim3(256), 0, c.stream, n, arr[k].get());
    CS_LAUNCH_CHECK();
    const f4v *r[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int k = 0; k < n_read; ++k) r[k] = arr[k].get();
    f4v *w = n_write ? arr[n_read].get() : nullptr;
    auto launch = [&]() {
        switch (n_read * 2 + n_write) {
#define CS_STREAM(NR, NW)                                                                                            \
    case NR * 2 + NW:                                                                                                \
        hipLaunchKernelGGL((k_stream<NR, NW>), dim3(G), dim3(256), 0, c.stream, n, r[0], r[1], r[2], r[3], w,       \
                           sink.get());                                                                              \
        break;
            CS_STREAM(0, 1)
            CS_STREAM(1, 0)
            CS_STREAM(1, 1)
            CS_STREAM(2, 0)
            CS_STREAM(2, 1)
            CS_STREAM(3, 0)
            CS_STREAM(3, 1)
            CS_STREAM(4, 0)
            CS_STREAM(4, 1)
#undef CS_STREAM
            default: break;
        }
        CS_LAUNCH_CHECK();
    };
    launch();   // warm-up
    hipEvent_t e0, e1;
    CS_HIP(hipEventCreate(&e0));
    CS_HIP(hipEventCreate(&e1));
    float ms = 0.0f;
    CS_HIP(hipEventRecord(e0, c.stream));
    for (int k = 0; k < reps; ++k) launch();
    CS_HIP(hipEventRecord(e1, c.stream));
    CS_HIP(hipEventSynchronize(e1));
    CS_HIP(hipEventElapsedTime(&ms, e0, e1));
    CS_HIP(hipEventDestroy(e0));
    CS_HIP(hipEventDestroy(e1));
    const double per = (double)ms / reps;   // ms per launch
    if (gbps) *gbps = (double)bytes * na / (per * 1e-3) / 1e9;
    if (us) *us = per * 1e3;
}

}  // namespace cs
