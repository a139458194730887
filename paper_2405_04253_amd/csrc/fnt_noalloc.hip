// fnt_cdc_aeq_batch_noalloc: the fused CDC + AEQ run of many channels with no
// allocation at all, for callers that cannot allocate device memory (code under
// graph capture, tight serving loops).
//
// fnt_plan_run with the fused schedule reads device tables and a work counter
// that fnt_plan_create allocates.  Here the tables and the counter live in a
// file-scope device array, `scratch`, of a fixed size (FNT_NOALLOC_MAX_CHANNELS
// channels): each GPU holds its own copy until the process ends.  The channel
// descriptors are read from device memory by a one-workgroup prepare kernel,
// which validates them, orders the channels longest chain first and writes the
// fused kernel's tables into `scratch`; the fused kernel then runs them.  Both
// launches go on the caller's stream, so the call also records into a graph
// under capture.  Every call on a GPU uses that GPU's one array: calls that
// overlap on one GPU (on different streams) race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "fnt_common.hpp"
#include "fnt_internal.hpp"

using namespace fnti;

namespace {

// Layout of `scratch`: the two work-counter words (kept at the start, in their
// own 256 bytes), the CDC table, the AEQ table, and one tap block that the
// entries of skipped channels point at.
constexpr size_t kMaxCh = FNT_NOALLOC_MAX_CHANNELS;
constexpr size_t kOffCdc = 256;
constexpr size_t kOffAeq = kOffCdc + ((kMaxCh * sizeof(CdcItem) + 255) & ~size_t(255));
constexpr size_t kOffDummy = kOffAeq + ((kMaxCh * sizeof(AeqItem) + 255) & ~size_t(255));
constexpr size_t kScratchBytes = kOffDummy + 512;
static_assert(kScratchBytes <= (size_t)FNT_NOALLOC_SCRATCH_BYTES, "scratch layout exceeds its stated size");

__device__ __align__(256) unsigned char scratch[FNT_NOALLOC_SCRATCH_BYTES];

__device__ __forceinline__ bool aligned_dev(const void *p, uintptr_t a) { return ((uintptr_t)p % a) == 0; }

// Whether descriptor d passes the checks fnt_plan_create makes on the host.
__device__ bool desc_valid(const fnt_channel_desc &d) {
    const fnt_cdc_params &c = d.cdc;
    const fnt_aeq_params &a = d.aeq;
    if (c.ntaps < 1 || c.ntaps > FNT_MAX_CDC_TAPS || c.requant_shift < 0 || c.requant_shift > 16 ||
        (c.decim_phase != 0 && c.decim_phase != 1))
        return false;
    for (int k = 0; k < c.ntaps; ++k)
        if (c.taps[k][0] < -32 || c.taps[k][0] > 31 || c.taps[k][1] < -32 || c.taps[k][1] > 31) return false;
    if (a.out_shift < 0 || a.out_shift > 24 || a.err_shift < 0 || a.err_shift > 62 || a.mu_shift < 0 ||
        a.mu_shift > 40 || a.const_unit < 1 || a.const_unit > 4096 || (a.update_enable != 0 && a.update_enable != 1) ||
        (a.gear_blocks > 0 && (a.mu_shift_late < 0 || a.mu_shift_late > 40)))
        return false;
    const uint64_t M = n_symbols(d.n, c.decim_phase);
    if (!d.taps || !aligned_dev(d.taps, 2) || (d.n > 0 && (!d.in || !aligned_dev(d.in, 4))) ||
        (M > 0 && (!d.out || !aligned_dev(d.out, 8))))
        return false;
    return true;
}

// One workgroup of 1024 threads: read and check the nch descriptors, sort them
// by AEQ chain length (longest first, ties in caller order; bitonic sort of
// 64-bit keys in LDS), write the fused kernel's tables, clear the work counter.
// A channel whose descriptor fails a check gets an empty entry (no input, no
// output, taps in the dummy block) at the end of the order and latches the
// parameter-error bit.
__global__ __launch_bounds__(1024) void noalloc_prepare_kernel(const fnt_channel_desc *descs, uint32_t nch,
                                                             unsigned char *sc, int *err) {
    __shared__ uint64_t key[kMaxCh];
    uint32_t np2 = 1;
    while (np2 < nch) np2 <<= 1;
    for (uint32_t i = threadIdx.x; i < np2; i += blockDim.x) {
        uint64_t k = 0;                                 // padding sorts last
        if (i < nch) {
            const fnt_channel_desc d = descs[i];
            const uint64_t blocks = desc_valid(d) ? (n_symbols(d.n, d.cdc.decim_phase) + 15) / 16 : 0;
            // key: 1 + chain length (42 bits), then the caller's index inverted so
            // that ties keep the caller's order under a descending sort
            const uint64_t capped = blocks < (1ull << 41) - 1 ? blocks : (1ull << 41) - 1;
            k = ((capped + 1) << 22) | (uint64_t)((1u << 22) - 1 - i);
        }
        key[i] = k;
    }
    __syncthreads();
    for (uint32_t size = 2; size <= np2; size <<= 1) {  // bitonic sort, descending
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = threadIdx.x; i < np2; i += blockDim.x) {
                const uint32_t j = i ^ stride;
                if (j > i) {
                    const bool desc = (i & size) == 0;
                    const uint64_t a = key[i], b = key[j];
                    if ((a < b) == desc) {
                        key[i] = b;
                        key[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    CdcItem *ct = reinterpret_cast<CdcItem *>(sc + kOffCdc);
    AeqItem *at = reinterpret_cast<AeqItem *>(sc + kOffAeq);
    int16_t *dummy = reinterpret_cast<int16_t *>(sc + kOffDummy);
    for (uint32_t k = threadIdx.x; k < nch; k += blockDim.x) {
        const uint32_t i = (1u << 22) - 1 - (uint32_t)(key[k] & ((1u << 22) - 1));
        const fnt_channel_desc d = descs[i];
        CdcItem c{};
        AeqItem a{};
        if (desc_valid(d)) {
            c.in = d.in;
            c.n = d.n;
            for (int t = 0; t < FNT_MAX_CDC_TAPS; ++t) {
                c.taps[t][0] = t < d.cdc.ntaps ? d.cdc.taps[t][0] : (int8_t)0;
                c.taps[t][1] = t < d.cdc.ntaps ? d.cdc.taps[t][1] : (int8_t)0;
            }
            c.ntaps = d.cdc.ntaps;
            c.shift = d.cdc.requant_shift;
            c.phase = d.cdc.decim_phase;
            a.m = n_symbols(d.n, d.cdc.decim_phase);
            a.taps = d.taps;
            a.out = d.out;
            a.out_shift = d.aeq.out_shift;
            a.err_shift = d.aeq.err_shift;
            a.mu_shift = d.aeq.mu_shift;
            a.mu_shift_late = d.aeq.gear_blocks > 0 ? d.aeq.mu_shift_late : d.aeq.mu_shift;
            a.gear_blocks = d.aeq.gear_blocks;
            a.const_unit = d.aeq.const_unit;
            a.update_enable = d.aeq.update_enable;
        } else {
            atomicOr(err, kFlagParam);
            c.ntaps = 1;
            a.taps = dummy;
            a.const_unit = 1;
        }
        ct[k] = c;
        at[k] = a;
    }
    if (threadIdx.x < 2) reinterpret_cast<uint32_t *>(sc)[threadIdx.x] = 0u;   // work counter
}

struct ScratchCtx {
    unsigned char *ptr = nullptr;   // this device's copy of `scratch`
    int grid_cap = 0;               // fused workgroups resident at once
};
std::mutex g_mu;
std::map<int, ScratchCtx> g_scratch;

// Set-up, once per device with that device current: the address of its copy of
// `scratch` (the array's name in host code is only a stand-in) and the fused
// kernel's residency.
int scratch_for_device(ScratchCtx *out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "noalloc: hipGetDevice");
    std::lock_guard<std::mutex> g(g_mu);
    ScratchCtx &c = g_scratch[dev];
    if (!c.ptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "noalloc: hipGetSymbolAddress(scratch)");
        c.ptr = static_cast<unsigned char *>(p);
        c.grid_cap = fused_capacity(4);
    }
    *out = c;
    return FNT_OK;
}

}  // namespace

extern "C" int fnt_cdc_aeq_batch_noalloc(const fnt_channel_desc *dev_channels, uint32_t nch, void *stream) {
    if (nch == 0) return FNT_OK;
    if (nch > FNT_NOALLOC_MAX_CHANNELS)
        return fail(FNT_E_INVAL, "noalloc: %u channels exceed the maximum of %u", nch,
                    (unsigned)FNT_NOALLOC_MAX_CHANNELS);
    if (!dev_channels || !aligned(dev_channels, 8)) return fail(FNT_E_INVAL, "noalloc: NULL or misaligned table");
    int *err = nullptr;
    int rc = device_err_flag(&err);
    if (rc) return rc;
    ScratchCtx c;
    if ((rc = scratch_for_device(&c))) return rc;
    hipStream_t s = (hipStream_t)stream;
    noalloc_prepare_kernel<<<1, 1024, 0, s>>>(dev_channels, nch, c.ptr, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "noalloc: prepare launch");
    const unsigned grid = (unsigned)std::min<uint32_t>(nch, c.grid_cap > 0 ? (uint32_t)c.grid_cap : 1024u);
    e = launch_fused(reinterpret_cast<const CdcItem *>(c.ptr + kOffCdc),
                     reinterpret_cast<const AeqItem *>(c.ptr + kOffAeq), (int)nch, CdcItem{}, AeqItem{}, 4,
                     reinterpret_cast<uint32_t *>(c.ptr), grid, (int)std::min<uint32_t>(nch, 512u), err, s);
    if (e != hipSuccess) return hip_fail(e, "noalloc: fused launch");
    return FNT_OK;
}
