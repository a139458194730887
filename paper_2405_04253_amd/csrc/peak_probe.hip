// Measured ceilings of one GPU for the roofline objects of the benchmark: the
// 32-bit integer VALU issue rate and the HBM copy bandwidth.  Not part of the
// receiver path; bench.py loads this library (libfntprobe.so) beside libfnt.so.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 16;     // independent chains per lane
constexpr int kUnroll = 16;     // instructions per chain per loop trip

// Each trip issues kChains * kUnroll instructions of one form (one lane-op per
// lane each), written as asm so the compiler neither folds nor reorders them.
// Form 0: v_add_u32 (issues at up to twice the base rate on this GPU); form 1:
// v_sub_u32 with SDWA word selects, the fold of the Fermat arithmetic (base
// rate, like shifts and 24-bit multiplies).
template <int FORM>
__global__ __launch_bounds__(256) void alu_probe_kernel(uint32_t *out, int trips) {
    uint32_t a[kChains];
    const uint32_t seed = threadIdx.x * 2654435761u + blockIdx.x;
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = seed + c;
    const uint32_t b = seed ^ 0x9E3779B9u;
    for (int t = 0; t < trips; ++t) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                if constexpr (FORM == 0)
                    __asm__ volatile("v_add_u32 %0, %0, %1" : "+v"(a[c]) : "v"(b));
                else
                    __asm__ volatile("v_sub_u32_sdwa %0, %0, %1 dst_sel:DWORD dst_unused:UNUSED_PAD "
                                     "src0_sel:WORD_0 src1_sel:WORD_1" : "+v"(a[c]) : "v"(b));
            }
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s ^= a[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void copy_probe_kernel(const uint4 *src, uint4 *dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

// 32-bit integer lane-operations per second of instruction form `form` (0: add,
// 1: SDWA subtract): `blocks` workgroups of 256 lanes, `trips` loop trips of 256
// instructions each; `out` is a device buffer of blocks * 256 uint32 (written,
// a sink for the results).  Returns 0, or -1 on a HIP error or another form.
int fntprobe_alu(int form, uint32_t *out, int blocks, int trips, double *lane_ops_per_s, void *stream) {
    if (form != 0 && form != 1) return -1;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1;
    auto launch = [&]() {
        if (form == 0) alu_probe_kernel<0><<<blocks, 256, 0, s>>>(out, trips);
        else alu_probe_kernel<1><<<blocks, 256, 0, s>>>(out, trips);
    };
    launch();                                                      // warm-up
    (void)hipEventRecord(e0, s);
    launch();
    (void)hipEventRecord(e1, s);
    hipError_t e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess || hipGetLastError() != hipSuccess || ms <= 0) return -1;
    *lane_ops_per_s = (double)blocks * 256.0 * trips * kUnroll * kChains / (ms * 1e-3);
    return 0;
}

// Device-to-device copy bandwidth (bytes read + bytes written per second) of a
// 16-byte-vector grid-stride copy of `bytes` (a multiple of 16) from src to dst.
int fntprobe_copy(const void *src, void *dst, size_t bytes, double *bytes_per_s, void *stream) {
    if (bytes % 16) return -1;
    hipStream_t s = (hipStream_t)stream;
    const size_t n = bytes / 16;
    const unsigned grid = 256 * 16;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1;
    copy_probe_kernel<<<grid, 256, 0, s>>>((const uint4 *)src, (uint4 *)dst, n);   // warm-up
    float best = 1e30f;
    for (int r = 0; r < 5; ++r) {
        (void)hipEventRecord(e0, s);
        copy_probe_kernel<<<grid, 256, 0, s>>>((const uint4 *)src, (uint4 *)dst, n);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) break;
        float ms = 0;
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (hipGetLastError() != hipSuccess || best >= 1e29f) return -1;
    *bytes_per_s = 2.0 * (double)bytes / (best * 1e-3);
    return 0;
}

}  // extern "C"
