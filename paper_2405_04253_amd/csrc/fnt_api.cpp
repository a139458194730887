// C ABI of libfnt: errors, parameter validation, single-stream calls and
// batched plans (device tables, hipGraph capture, schedule autotuning).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "fnt_common.hpp"
#include "fnt_internal.hpp"

using namespace fnti;

namespace fnti {

static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(FNT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// The per-device error flag is a device variable (each GPU holds its own copy,
// zero at load), so no call ever allocates it; host code uses the address
// hipGetSymbolAddress gives for the current device, never the variable's name.
__device__ int g_fnt_err_flag;

struct DeviceCtx {
    int *d_err = nullptr;
};
static std::mutex g_ctx_mu;
static std::map<int, DeviceCtx> g_ctx;
int device_err_flag(int **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> g(g_ctx_mu);
    DeviceCtx &c = g_ctx[dev];
    if (!c.d_err) {
        e = hipGetSymbolAddress((void **)&c.d_err, HIP_SYMBOL(g_fnt_err_flag));
        if (e != hipSuccess) {
            c.d_err = nullptr;
            return hip_fail(e, "hipGetSymbolAddress(error flag)");
        }
    }
    *out = c.d_err;
    return FNT_OK;
}
int validate_cdc(const fnt_cdc_params *p) {
    if (!p) return fail(FNT_E_INVAL, "cdc params: NULL");
    if (p->ntaps < 1 || p->ntaps > FNT_MAX_CDC_TAPS)
        return fail(FNT_E_INVAL, "cdc params: ntaps %d outside [1, 32]", p->ntaps);
    if (p->requant_shift < 0 || p->requant_shift > 16)
        return fail(FNT_E_INVAL, "cdc params: requant_shift %d outside [0, 16]", p->requant_shift);
    if (p->decim_phase != 0 && p->decim_phase != 1)
        return fail(FNT_E_INVAL, "cdc params: decim_phase %d not 0 or 1", p->decim_phase);
    for (int k = 0; k < p->ntaps; ++k)
        for (int c = 0; c < 2; ++c)
            if (p->taps[k][c] < -32 || p->taps[k][c] > 31)
                return fail(FNT_E_RANGE, "cdc params: tap %d component %d = %d outside 6 bit", k, c,
                            p->taps[k][c]);
    return FNT_OK;
}

int validate_aeq(const fnt_aeq_params *p) {
    if (!p) return fail(FNT_E_INVAL, "aeq params: NULL");
    if (p->out_shift < 0 || p->out_shift > 24)
        return fail(FNT_E_INVAL, "aeq params: out_shift %d outside [0, 24]", p->out_shift);
    if (p->err_shift < 0 || p->err_shift > 62)
        return fail(FNT_E_INVAL, "aeq params: err_shift %d outside [0, 62]", p->err_shift);
    if (p->mu_shift < 0 || p->mu_shift > 40)
        return fail(FNT_E_INVAL, "aeq params: mu_shift %d outside [0, 40]", p->mu_shift);
    if (p->gear_blocks > 0 && (p->mu_shift_late < 0 || p->mu_shift_late > 40))
        return fail(FNT_E_INVAL, "aeq params: mu_shift_late %d outside [0, 40]", p->mu_shift_late);
    if (p->const_unit < 1 || p->const_unit > 4096)
        return fail(FNT_E_INVAL, "aeq params: const_unit %d outside [1, 4096]", p->const_unit);
    if (p->update_enable != 0 && p->update_enable != 1)
        return fail(FNT_E_INVAL, "aeq params: update_enable %d not 0 or 1", p->update_enable);
    return FNT_OK;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

void fill_cdc_item(CdcItem &it, const int8_t *in, uint64_t n, const fnt_cdc_params *p) {
    std::memset(&it, 0, sizeof it);
    it.in = in;
    it.n = n;
    std::memcpy(it.taps, p->taps, sizeof it.taps);
    for (int k = p->ntaps; k < FNT_MAX_CDC_TAPS; ++k) it.taps[k][0] = it.taps[k][1] = 0;
    it.ntaps = p->ntaps;
    it.shift = p->requant_shift;
    it.phase = p->decim_phase;
}

void fill_aeq_item(AeqItem &it, const int8_t *a, uint64_t m, int16_t *taps, const fnt_aeq_params *p,
                   int16_t *out) {
    std::memset(&it, 0, sizeof it);
    it.a = a;
    it.m = m;
    it.taps = taps;
    it.out = out;
    it.out_shift = p->out_shift;
    it.err_shift = p->err_shift;
    it.mu_shift = p->mu_shift;
    it.const_unit = p->const_unit;
    it.update_enable = p->update_enable;
    it.mu_shift_late = p->gear_blocks > 0 ? p->mu_shift_late : p->mu_shift;
    it.gear_blocks = p->gear_blocks;
    it.block0 = 0;
}

// Default CDC schedule: the lane-per-block kernel (blocks_per_wave = 0), four
// waves per workgroup.
void default_cdc_schedule(uint64_t total_blocks, int *wpg, int *bpw) {
    (void)total_blocks;
    *wpg = 4;
    *bpw = 0;
}

// Launch the CDC with a schedule (wpg, bpw): bpw = 0 is the lane-per-block
// kernel, bpw >= 1 the wave-per-block kernel with bpw consecutive blocks per
// wave.  The exact output z only exists in the wave-per-block kernel, which then
// runs with enough waves to fill 256 CUs several times over.
hipError_t run_cdc(const CdcItem *items, int nitems, const CdcItem &single, uint64_t blocks,
                   uint64_t chunks, int wpg, int bpw, bool with_z, int *err, hipStream_t s) {
    if (bpw == 0 && !with_z) return launch_cdc(items, nitems, single, blocks, chunks, 0, wpg, 1, false, err, s);
    const int b = bpw ? bpw : (int)std::max<uint64_t>(1, std::min<uint64_t>(64, blocks / (256ull * 4 * 16)));
    return launch_cdc(items, nitems, single, blocks, chunks, 1, wpg, b, with_z, err, s);
}

}  // namespace fnti

// ------------------------------------------------------------------ C ABI --

extern "C" {

const char *fnt_last_error(void) { return fnti::g_last_error.c_str(); }

int fnt_version(void) { return 10000; }

int fnt_check(void *stream) {
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    int *d = nullptr;
    int rc = device_err_flag(&d);
    if (rc) return rc;
    int h = 0;
    e = hipMemcpy(&h, d, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(range flag)");
    if (h) {
        e = hipMemset(d, 0, sizeof(int));
        if (e != hipSuccess) return hip_fail(e, "hipMemset(range flag)");
        if (h & kFlagStall)
            return fail(FNT_E_DEVICE, "a bounded wait of a fused launch gave up (flags 0x%x)", h);
        if (h & kFlagParam)
            return fail(FNT_E_INVAL, "a device-side channel descriptor was invalid; its channel was skipped "
                                     "(flags 0x%x)", h);
        return fail(FNT_E_RANGE, "input value outside its declared width (flags 0x%x)", h);
    }
    return FNT_OK;
}

static int transform_common(const uint32_t *x, uint32_t *X, size_t batch, int t, int log2n,
                            int alpha_kind, bool inv, void *stream) {
    // t in {2, 3, 4}; N is the radix's order: 2^(t+1) for alpha = 2, 2^(t+2) for sqrt 2
    const bool legal = t >= 2 && t <= 4 &&
                       ((alpha_kind == FNT_ALPHA_2 && log2n == t + 1) ||
                        (alpha_kind == FNT_ALPHA_SQRT2 && log2n == t + 2));
    if (!legal)
        return fail(FNT_E_INVAL, "unsupported transform (t=%d, log2n=%d, alpha=%d)", t, log2n,
                    alpha_kind);
    if (batch == 0) return FNT_OK;
    if (!x || !X) return fail(FNT_E_INVAL, "transform: NULL buffer");
    if (!aligned(x, 4) || !aligned(X, 4)) return fail(FNT_E_INVAL, "transform: misaligned buffer");
    int *err = nullptr;
    int rc = device_err_flag(&err);
    if (rc) return rc;
    hipError_t e = launch_transform(x, X, batch, t, log2n, alpha_kind, inv, err, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "transform launch");
    return FNT_OK;
}

int fnt_forward(const uint32_t *x, uint32_t *X, size_t batch, int t, int log2n, int alpha_kind,
                void *stream) {
    return transform_common(x, X, batch, t, log2n, alpha_kind, false, stream);
}

int fnt_inverse(const uint32_t *X, uint32_t *x, size_t batch, int t, int log2n, int alpha_kind,
                void *stream) {
    return transform_common(X, x, batch, t, log2n, alpha_kind, true, stream);
}

int fnt_cdc(const int8_t *in, uint64_t n, const fnt_cdc_params *p, int32_t *out_exact,
            int8_t *out_1sps, void *stream) {
    int rc = validate_cdc(p);
    if (rc) return rc;
    if (n == 0) return FNT_OK;
    if (!in) return fail(FNT_E_INVAL, "fnt_cdc: NULL input");
    if (!aligned(in, 4) || (out_exact && !aligned(out_exact, 16)) || (out_1sps && !aligned(out_1sps, 4)))
        return fail(FNT_E_INVAL, "fnt_cdc: misaligned buffer");
    int *err = nullptr;
    if ((rc = device_err_flag(&err))) return rc;
    CdcItem it;
    fill_cdc_item(it, in, n, p);
    it.z_out = out_exact;
    it.a_out = out_1sps;
    int wpg, bpw;
    default_cdc_schedule(cdc_blocks(n), &wpg, &bpw);
    hipError_t e = run_cdc(nullptr, 0, it, cdc_blocks(n), cdc_chunks(n), wpg, bpw, out_exact != nullptr, err,
                           (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fnt_cdc launch");
    return FNT_OK;
}

int fnt_aeq(const int8_t *in_1sps, uint64_t m, int16_t *taps, const fnt_aeq_params *p, int16_t *out,
            void *stream) {
    int rc = validate_aeq(p);
    if (rc) return rc;
    if (!taps) return fail(FNT_E_INVAL, "fnt_aeq: NULL taps");
    if (m > 0 && (!in_1sps || !out)) return fail(FNT_E_INVAL, "fnt_aeq: NULL buffer");
    if (!aligned(in_1sps, 4) || !aligned(out, 8) || !aligned(taps, 2))
        return fail(FNT_E_INVAL, "fnt_aeq: misaligned buffer");
    int *err = nullptr;
    if ((rc = device_err_flag(&err))) return rc;
    AeqItem it;
    fill_aeq_item(it, in_1sps, m, taps, p, out);
    hipError_t e = launch_aeq(nullptr, 0, it, 0, 4, err, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fnt_aeq launch");
    return FNT_OK;
}

// AEQ lanes per transform of the single-stream fused launch.
constexpr int kSingleLpt = 16;

int fnt_cdc_aeq(const int8_t *in, uint64_t n, const fnt_cdc_params *cp, int16_t *taps,
                const fnt_aeq_params *ap, int16_t *out, void *stream) {
    int rc = validate_cdc(cp);
    if (rc) return rc;
    if ((rc = validate_aeq(ap))) return rc;
    if (!taps) return fail(FNT_E_INVAL, "fnt_cdc_aeq: NULL taps");
    const uint64_t M = n_symbols(n, cp->decim_phase);
    if ((n > 0 && !in) || (M > 0 && !out)) return fail(FNT_E_INVAL, "fnt_cdc_aeq: NULL buffer");
    if (!aligned(in, 4) || !aligned(out, 8) || !aligned(taps, 2))
        return fail(FNT_E_INVAL, "fnt_cdc_aeq: misaligned buffer");
    int *err = nullptr;
    if ((rc = device_err_flag(&err))) return rc;
    // one launch of the fused kernel, one workgroup per polarisation half: in
    // each, producer waves run the CDC chunk by chunk into LDS while four waves
    // run the half's AEQ chain (the shortest serial latency per block on an
    // otherwise idle GPU)
    CdcItem ci;
    fill_cdc_item(ci, in, n, cp);
    AeqItem ai;
    fill_aeq_item(ai, nullptr, M, taps, ap, out);
    hipError_t e = launch_fused(nullptr, nullptr, 1, ci, ai, kSingleLpt, nullptr, fused_split_grid(1), 1, err,
                                (hipStream_t)stream, true);
    if (e != hipSuccess) return hip_fail(e, "fnt_cdc_aeq: launch");
    return FNT_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ plans --

struct fnt_plan {
    int device = 0;
    std::vector<CdcItem> cdc_host;
    std::vector<AeqItem> aeq_host;
    CdcItem *cdc_dev = nullptr;
    AeqItem *aeq_dev = nullptr;
    int8_t *abuf = nullptr;
    int *err = nullptr;
    uint64_t total_blocks = 0, total_chunks = 0;
    fnt_plan_info info{};
    int wpg = 4, bpw = 0, variant = 0, wpp = 1;   // CDC: bpw = 0 is the lane-per-block kernel
    int cdc_variant = 0;                          // 1: direct time-domain comparator
    // AEQ split: the n_long longest chains (table prefix) run with wpp_long waves
    // per half in a launch concurrent with the rest
    int wpp_long = 4;
    size_t n_long = 0;
    // pipelined lead: the n_lead longest channels' CDC first, their AEQ on the side
    // stream concurrently with the others' CDC and AEQ; the n_top longest of them
    // may form a first level of their own (CDC first of all, AEQ on side2).
    // cdc_seg_dev is the CDC table with each segment [0, top), [top, lead),
    // [lead, n) rebased to block 0 / chunk 0, built for (seg_top, seg_lead)
    size_t n_lead = 0, n_top = 0, seg_lead = 0, seg_top = 0;
    int lead_form = -1, top_form = -1;  // AEQ forms of the levels (-1: the long chains' form)
    CdcItem *cdc_seg_dev = nullptr;
    hipStream_t side = nullptr;        // second stream for the concurrent AEQ launch
    hipStream_t side2 = nullptr;       // third stream: the first lead level
    hipEvent_t fork = nullptr, join = nullptr, fork2 = nullptr, join2 = nullptr;
    hipEvent_t tev[8] = {};            // fnt_plan_run_timed
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // fused persistent CDC + AEQ (one launch per run; fused_lpt = 0: off): AEQ
    // lanes per transform, channels at raised priority, workgroups, and the two
    // work-counter words the kernel takes channels from (zero between launches)
    int fused_lpt = 0;
    bool fused_split = false;        // one workgroup per polarisation half
    size_t fused_prio = 0;
    unsigned fused_grid = 0;
    uint32_t *queue = nullptr;
};

// The CDC of the table `tab` (nitems items whose block0 / chunk0 start at 0).
static hipError_t plan_cdc(fnt_plan *p, const CdcItem *tab, int nitems, uint64_t blocks, uint64_t chunks,
                           hipStream_t s) {
    return p->cdc_variant == 1 ? launch_cdc(tab, nitems, CdcItem{}, blocks, chunks, 2, p->wpg, 1, false, p->err, s)
                               : run_cdc(tab, nitems, CdcItem{}, blocks, chunks, p->wpg, p->bpw, false, p->err, s);
}

static int plan_launch_cdc(fnt_plan *p, hipStream_t s) {
    hipError_t e = plan_cdc(p, p->cdc_dev, (int)p->cdc_host.size(), p->total_blocks, p->total_chunks, s);
    if (e != hipSuccess) return hip_fail(e, "plan: cdc launch");
    return FNT_OK;
}

// The AEQ of the items [first, n) of the longest-first table, of which the
// first nl run in the long chains' form: one launch on s when possible.
static bool plan_aeq_one_launch(const fnt_plan *p, int nl, int count) {
    return p->variant != 0 || nl == 0 || nl >= count || aeq_split_fusable(p->wpp_long, p->wpp);
}

static hipError_t plan_aeq_range(fnt_plan *p, int first, int nl, int count, hipStream_t s) {
    const AeqItem *items = p->aeq_dev + first;
    if (p->variant != 0 || nl == 0 || nl >= count) {
        const int w = (p->variant == 0 && nl >= count) ? p->wpp_long : p->wpp;
        return launch_aeq(items, count, AeqItem{}, p->variant, w, p->err, s);
    }
    return launch_aeq_split(items, nl, count, p->wpp_long, p->wpp, p->err, s);   // long chains dispatched first
}

// Lead channels in effect for the plan's current schedule (0: none), and the
// first level's channels among them (0: one level).
// Lead form kFusedLead: the lead channels run as one launch of the fused CDC +
// AEQ kernel (one wave per half) on the side stream, with no CDC of their own
// before it, so their chains start at once.
constexpr int kFusedLead = 6;

static size_t plan_top(const fnt_plan *p) {
    if (p->variant == 0 && p->lead_form == kFusedLead) return 0;   // a fused lead has no first level
    return p->n_top > 0 && p->n_top < p->n_lead ? p->n_top : 0;
}

// AEQ forms of the lead after its first level, and of the first level
static int lead_form_of(const fnt_plan *p) { return p->lead_form >= 0 ? p->lead_form : p->wpp_long; }
static bool lead_is_fused(const fnt_plan *p) { return p->variant == 0 && lead_form_of(p) == kFusedLead; }
static int top_form_of(const fnt_plan *p) { return p->top_form >= 0 ? p->top_form : p->wpp_long; }

// A first level whose form pairs with the lead's in one split launch runs inside
// the lead's launch (no CDC segment, stream or launch of its own).
static bool plan_top_fused(const fnt_plan *p) {
    return plan_top(p) > 0 && p->variant == 0 && !lead_is_fused(p) && aeq_split_fusable(top_form_of(p), lead_form_of(p));
}
// The first level's own CDC segment (0 when there is none or it is fused).
static size_t plan_cdc_top(const fnt_plan *p) { return plan_top_fused(p) ? 0 : plan_top(p); }

static size_t plan_lead(const fnt_plan *p) {
    const size_t n = p->aeq_host.size();
    if (p->fused_lpt) return 0;                        // the fused kernel runs every channel
    if (p->n_lead == 0 || p->n_lead >= n || p->seg_lead != p->n_lead ||
        p->seg_top != plan_cdc_top(p) || !p->cdc_seg_dev)
        return 0;
    const size_t rest_long = p->n_long > p->n_lead ? p->n_long - p->n_lead : 0;
    return plan_aeq_one_launch(p, (int)rest_long, (int)(n - p->n_lead)) ? p->n_lead : 0;
}

static uint64_t aeq_blocks_of(const fnt_plan *p, size_t lo, size_t hi) {
    uint64_t b = 0;
    for (size_t i = lo; i < hi; ++i) b += (p->aeq_host[i].m + 15) / 16;
    return b;
}

static int plan_launch_aeq(fnt_plan *p, hipStream_t s, hipStream_t side) {
    const int n = (int)p->aeq_host.size();
    const int nl = (int)std::min<size_t>(p->n_long, (size_t)n);
    hipError_t e;
    if (plan_aeq_one_launch(p, nl, n)) {
        e = plan_aeq_range(p, 0, nl, n, s);
        if (e != hipSuccess) return hip_fail(e, "plan: aeq launch");
        return FNT_OK;
    }
    e = hipEventRecord(p->fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, p->fork, 0);
    if (e == hipSuccess) e = launch_aeq(p->aeq_dev, nl, AeqItem{}, 0, p->wpp_long, p->err, s, true);
    if (e == hipSuccess) e = launch_aeq(p->aeq_dev + nl, n - nl, AeqItem{}, 0, p->wpp, p->err, side);
    if (e == hipSuccess) e = hipEventRecord(p->join, side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, p->join, 0);
    if (e != hipSuccess) return hip_fail(e, "plan: aeq launch");
    return FNT_OK;
}

// Launch sequence of a plan on stream s.  Without a lead: the CDC over all
// blocks, then the AEQ (one launch, or the long chains on s concurrently with
// the others on the side stream).  With a lead of L channels: the CDC of the L
// longest channels; fork; their AEQ on the side stream; the CDC of the others
// and their AEQ on s; join.  With a first level of T < L channels: the CDC of
// the T longest; fork; their AEQ on side2; then as above for channels [T, L).
// Fork / join are events, which a graph capture turns into parallel branches.
// `ev` (timing, direct launches only) receives start, CDC end, lead AEQ start,
// lead AEQ end, AEQ end, done, first-level AEQ start and end.
static unsigned plan_fused_grid(const fnt_plan *p, int lpt, bool split) {
    const size_t n = p->aeq_host.size();
    if (split) return fused_split_grid((int)n);
    const int cap = fused_capacity(lpt);
    return (unsigned)std::min<size_t>(n, cap > 0 ? (size_t)cap : 1024);
}

static int plan_launch(fnt_plan *p, hipStream_t s, hipStream_t side, hipStream_t side2,
                       hipEvent_t *ev = nullptr) {
    auto rec = [&](int i, hipStream_t st) { return ev ? hipEventRecord(ev[i], st) : hipSuccess; };
    hipError_t e = rec(0, s);
    if (p->fused_lpt) {
        // one launch: every channel's CDC and AEQ in the fused persistent kernel
        if (e == hipSuccess) e = rec(1, s);
        if (e == hipSuccess)
            e = launch_fused(p->cdc_dev, p->aeq_dev, (int)p->aeq_host.size(), CdcItem{}, AeqItem{}, p->fused_lpt,
                             p->fused_split ? nullptr : p->queue, p->fused_grid,
                             (int)std::min<size_t>(p->fused_prio, 1u << 26), p->err, s, p->fused_split);
        if (e == hipSuccess) e = rec(4, s);
        if (e == hipSuccess) e = rec(5, s);
        if (e != hipSuccess) return hip_fail(e, "plan: fused launch");
        return FNT_OK;
    }
    const size_t lead = plan_lead(p);
    const bool fused = lead && plan_top_fused(p);
    const size_t top = lead && !fused ? plan_top(p) : 0;      // a first level of its own
    if (lead == 0) {
        int rc = e == hipSuccess ? plan_launch_cdc(p, s) : hip_fail(e, "plan: timing event");
        if (!rc && (e = rec(1, s)) != hipSuccess) rc = hip_fail(e, "plan: timing event");
        if (!rc) rc = plan_launch_aeq(p, s, side);
        if (!rc && (e = rec(4, s)) != hipSuccess) rc = hip_fail(e, "plan: timing event");
        if (!rc && (e = rec(5, s)) != hipSuccess) rc = hip_fail(e, "plan: timing event");
        return rc;
    }
    const size_t n = p->aeq_host.size();
    const int rest_long = (int)(p->n_long > lead ? p->n_long - lead : 0);
    // the CDC of the segment [a, b) from the rebased table
    auto seg_cdc = [&](size_t a, size_t b) {
        const CdcItem &ca = p->cdc_host[a];
        const uint64_t blocks = (b < n ? p->cdc_host[b].block0 : p->total_blocks) - ca.block0;
        const uint64_t chunks = (b < n ? p->cdc_host[b].chunk0 : p->total_chunks) - ca.chunk0;
        return plan_cdc(p, p->cdc_seg_dev + a, (int)(b - a), blocks, chunks, s);
    };
    const int lf = lead_form_of(p);
    const int tf = top_form_of(p);
    bool cdc_enqueued = false;                 // the others' CDC segment [lead, n)
    if (top) {                                 // the first level's CDC, then fork (its AEQ below)
        if (e == hipSuccess) e = seg_cdc(0, top);
        if (e == hipSuccess) e = hipEventRecord(p->fork2, s);
    }
    if (lead_is_fused(p)) {
        // the lead's CDC and AEQ in one fused launch on the side stream, at once
        if (e == hipSuccess) e = hipEventRecord(p->fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(side, p->fork, 0);
        if (e == hipSuccess) e = rec(2, side);
        if (e == hipSuccess)
            e = launch_fused(p->cdc_dev, p->aeq_dev, (int)lead, CdcItem{}, AeqItem{}, 4, p->queue,
                             (unsigned)std::min<size_t>(lead, std::max(1, fused_capacity(4))), (int)lead, p->err,
                             side);
        if (e == hipSuccess) e = rec(3, side);
    } else if (e == hipSuccess) {
        e = seg_cdc(top, lead);
    }
    if (top) {
        // the first level's AEQ after the lead's CDC is enqueued (CDC workgroups
        // dispatch ahead of the long-lived AEQ waves, as for the lead below)
        if (e == hipSuccess) e = hipStreamWaitEvent(side2, p->fork2, 0);
        if (e == hipSuccess) e = rec(6, side2);
        if (e == hipSuccess) e = launch_aeq(p->aeq_dev, (int)top, AeqItem{}, p->variant, tf, p->err, side2, true);
        if (e == hipSuccess) e = rec(7, side2);
    }
    if (lead_is_fused(p)) {
    } else if (fused) {
        // the first level's chains first in the lead's own split launch
        if (e == hipSuccess) e = hipEventRecord(p->fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(side, p->fork, 0);
        if (e == hipSuccess) e = rec(2, side);
        if (e == hipSuccess)
            e = launch_aeq_split(p->aeq_dev, (int)plan_top(p), (int)lead, tf, lf, p->err, side, true);
        if (e == hipSuccess) e = rec(3, side);
    } else if (e == hipSuccess) {
        // The others' CDC is enqueued before the lead's AEQ, which waits for the
        // lead's CDC only (the fork event is recorded before the others' CDC).
        // Graph replays dispatch the nodes in this order; with the lead's AEQ
        // first, its long-lived waves took the compute units ahead of the short
        // CDC workgroups and the others' CDC ran twice as long.
        e = hipEventRecord(p->fork, s);
        if (e == hipSuccess) e = seg_cdc(lead, n);
        if (e == hipSuccess) e = hipStreamWaitEvent(side, p->fork, 0);
        if (e == hipSuccess) e = rec(2, side);
        if (e == hipSuccess)
            e = launch_aeq(p->aeq_dev + top, (int)(lead - top), AeqItem{}, p->variant, lf, p->err, side, true);
        if (e == hipSuccess) e = rec(3, side);
        cdc_enqueued = true;
    }
    if (e == hipSuccess && !cdc_enqueued) e = seg_cdc(lead, n);
    if (e == hipSuccess) e = rec(1, s);
    if (e == hipSuccess) e = plan_aeq_range(p, (int)lead, rest_long, (int)(n - lead), s);
    if (e == hipSuccess) e = rec(4, s);
    if (e == hipSuccess) e = hipEventRecord(p->join, side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, p->join, 0);
    if (top) {
        if (e == hipSuccess) e = hipEventRecord(p->join2, side2);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, p->join2, 0);
    }
    if (e == hipSuccess) e = rec(5, s);
    if (e != hipSuccess) return hip_fail(e, "plan: pipelined launch");
    return FNT_OK;
}

// Upload the CDC table with the segments [0, top), [top, lead), [lead, n) each
// rebased to start at block 0 and chunk 0 (synchronous on s); top = 0: two
// segments.  lead = 0 or >= n: no lead, nothing to build.
static int plan_build_segments(fnt_plan *p, size_t top, size_t lead, hipStream_t s) {
    const size_t n = p->cdc_host.size();
    if (lead == 0 || lead >= n) {
        p->seg_lead = p->seg_top = 0;
        return FNT_OK;
    }
    if (top >= lead) top = 0;
    hipError_t e = hipSuccess;
    if (!p->cdc_seg_dev) e = hipMalloc(&p->cdc_seg_dev, n * sizeof(CdcItem));
    if (e != hipSuccess) return fail(FNT_E_NOMEM, "plan: lead table: %s", hipGetErrorString(e));
    std::vector<CdcItem> tab(p->cdc_host);
    for (size_t i = 0; i < n; ++i) {
        const CdcItem &first = p->cdc_host[i < top ? 0 : i < lead ? top : lead];
        tab[i].block0 -= first.block0;
        tab[i].chunk0 -= first.chunk0;
    }
    e = hipMemcpyAsync(p->cdc_seg_dev, tab.data(), n * sizeof(CdcItem), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "plan: upload lead table");
    p->seg_lead = lead;
    p->seg_top = top;
    return FNT_OK;
}

static void plan_drop_graph(fnt_plan *p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

static int plan_capture(fnt_plan *p, hipStream_t s) {
    plan_drop_graph(p);
    hipStream_t cs = nullptr, cs2 = nullptr, cs3 = nullptr;
    auto drop = [&]() {
        if (cs) (void)hipStreamDestroy(cs);
        if (cs2) (void)hipStreamDestroy(cs2);
        if (cs3) (void)hipStreamDestroy(cs3);
    };
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs3, hipStreamNonBlocking);
    if (e != hipSuccess) {
        drop();
        return hip_fail(e, "plan: capture streams");
    }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        drop();
        return hip_fail(e, "plan: begin capture");
    }
    int rc = plan_launch(p, cs, cs2, cs3);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    drop();
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "plan: end capture");
    e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "plan: graph instantiate");
    }
    p->graph = g;
    (void)s;
    return FNT_OK;
}

constexpr int kTuneVersion = 9;

static std::string tune_key(const fnt_plan *p) {
    // length histogram (log2 buckets of instants) + channel count + variant
    int hist[48] = {0};
    for (const CdcItem &c : p->cdc_host) {
        int b = 0;
        while (b < 47 && (1ull << (b + 1)) <= c.n) ++b;
        hist[b]++;
    }
    std::ostringstream k;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) k << prop.gcnArchName;
    // the schedule vocabulary (CDC mappings, AEQ forms, split rules) is versioned
    // so that entries written by a build with other meanings are not reused
    k << "|s" << kTuneVersion << "|v" << p->variant << "|ch" << p->cdc_host.size() << "|";
    for (int i = 0; i < 48; ++i)
        if (hist[i]) k << i << ":" << hist[i] << ",";
    return k.str();
}

// The last entry for `key`; the values are range-checked by the caller.
static bool tune_cache_lookup(const char *path, const std::string &key, int *wpg, int *bpw, int *wpp,
                              int *wpp_long, long long *n_long, long long *n_lead, int *lead_form,
                              long long *n_top, int *top_form, int *fused_lpt, long long *fused_prio) {
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        // one JSON object per line: {"key": "...", "wpg": W, "bpw": B, ...}
        size_t a = line.find("\"key\": \"");
        if (a == std::string::npos) continue;
        size_t b = line.find('"', a + 8);
        if (b == std::string::npos || line.substr(a + 8, b - a - 8) != key) continue;
        int w = 0, bb = 0, pp = 0;
        size_t pw = line.find("\"wpg\": "), pb = line.find("\"bpw\": "), pq = line.find("\"wpp\": ");
        if (pw == std::string::npos || pb == std::string::npos || pq == std::string::npos) continue;
        w = std::atoi(line.c_str() + pw + 7);
        bb = std::atoi(line.c_str() + pb + 7);
        pp = std::atoi(line.c_str() + pq + 7);
        size_t pl = line.find("\"wpp_long\": "), pn = line.find("\"n_long\": "),
               pd = line.find("\"n_lead\": "), pf = line.find("\"lead_form\": "),
               pt = line.find("\"n_top\": "), ptf = line.find("\"top_form\": ");
        size_t pfl = line.find("\"fused_lpt\": "), pfp = line.find("\"fused_prio\": ");
        if (pl == std::string::npos || pn == std::string::npos || pd == std::string::npos ||
            pf == std::string::npos || pt == std::string::npos || ptf == std::string::npos ||
            pfl == std::string::npos || pfp == std::string::npos)
            continue;
        *fused_lpt = std::atoi(line.c_str() + pfl + 13);
        *fused_prio = std::atoll(line.c_str() + pfp + 14);
        *wpg = w;
        *bpw = bb;
        *wpp = pp;
        *wpp_long = std::atoi(line.c_str() + pl + 12);
        *n_long = std::atoll(line.c_str() + pn + 10);
        *n_lead = std::atoll(line.c_str() + pd + 10);
        *lead_form = std::atoi(line.c_str() + pf + 13);
        *n_top = std::atoll(line.c_str() + pt + 9);
        *top_form = std::atoi(line.c_str() + ptf + 12);
        found = true;
    }
    return found;
}

static void tune_cache_store(const char *path, const std::string &key, int wpg, int bpw, int wpp,
                             int wpp_long, long long n_long, long long n_lead, int lead_form, long long n_top,
                             int top_form, int fused_lpt, long long fused_prio, double ms) {
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    f << "{\"key\": \"" << key << "\", \"wpg\": " << wpg << ", \"bpw\": " << bpw << ", \"wpp\": " << wpp
      << ", \"wpp_long\": " << wpp_long << ", \"n_long\": " << n_long << ", \"n_lead\": " << n_lead
      << ", \"lead_form\": " << lead_form << ", \"n_top\": " << n_top << ", \"top_form\": " << top_form
      << ", \"fused_lpt\": " << fused_lpt << ", \"fused_prio\": " << fused_prio << ", \"ms\": " << ms << "}\n";
}

// Default AEQ schedule: with few channels the chip is idle, so spread each
// polarisation half over more waves to shorten the serial chain.
// AEQ forms of a plan (the `waves per half` value): 0 = one transform per lane
// (two channels per wave), 3 = two lanes per transform (one channel per wave),
// 1 / 2 / 4 = split by output polarisation with that many waves per half, 5 =
// split by output polarisation with both halves in one workgroup.
// Cost per block rises, and the serial latency per block falls, in this order.
static bool valid_form(int f) { return f >= 0 && f <= 5; }
static int form_rank(int f) { return f == 0 ? 0 : f == 3 ? 1 : (f == 1 || f == 5) ? 2 : f == 2 ? 3 : 4; }
static int default_wpp(size_t nch) { return nch >= 512 ? 3 : (nch >= 128 ? 2 : 4); }

static int plan_autotune(fnt_plan *p, hipStream_t s, const char *cache, bool quick) {
    std::string key = tune_key(p) + (quick ? "|quick" : "");
    int w, b, q, ql, lf, tf, fl;
    long long nl, nd, nt, fp;
    if (tune_cache_lookup(cache, key, &w, &b, &q, &ql, &nl, &nd, &lf, &nt, &tf, &fl, &fp) &&
        (w == 1 || w == 2 || w == 4) &&
        b >= 0 && b <= 1024 && valid_form(q) && valid_form(ql) && nl >= 0 && nd >= 0 &&
        (size_t)nd < std::max<size_t>(1, p->aeq_host.size()) && (lf == -1 || lf == kFusedLead || valid_form(lf)) && nt >= 0 &&
        (nt == 0 || nt < nd) && (tf == -1 || valid_form(tf)) &&
        (fl == 0 || std::abs(fl) == 4 || std::abs(fl) == 8 || std::abs(fl) == 16) && fp >= 0) {
        p->fused_lpt = std::abs(fl);
        p->fused_split = fl < 0;
        p->fused_prio = (size_t)fp;
        if (fl) p->fused_grid = plan_fused_grid(p, fl, p->fused_split);
        p->wpg = w;
        p->bpw = b;
        p->wpp = q;
        p->wpp_long = ql;
        p->n_long = (size_t)nl;
        p->n_lead = (size_t)nd;
        p->lead_form = lf;
        p->n_top = (size_t)nt;
        p->top_form = tf;
        return FNT_OK;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(FNT_E_DEVICE, "plan: autotune events");
    int reps = 2;
    auto time_it = [&](auto &&launch) -> double {
        float ms = 0, best = 1e30f;
        for (int rep = 0; rep < reps; ++rep) {
            (void)hipEventRecord(e0, s);
            if (launch() != hipSuccess) return 1e30;
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            (void)hipEventElapsedTime(&ms, e0, e1);
            best = std::min(best, ms);
        }
        return best;
    };
    // CDC schedules
    double best_cdc = 1e30;
    int bw = p->wpg, bb = p->bpw;
    for (int wpg : {1, 2, 4})
        for (int bpw : {0, 1, 4, 16, 64}) {
            if ((uint64_t)bpw > std::max<uint64_t>(1, p->total_blocks)) continue;
            if (quick && bpw != 0) continue;            // quick: the lane-per-block groupings only
            double ms = time_it([&] {
                return run_cdc(p->cdc_dev, (int)p->cdc_host.size(), CdcItem{}, p->total_blocks, p->total_chunks,
                               wpg, bpw, false, p->err, s);
            });
            if (ms < best_cdc) {
                best_cdc = ms;
                bw = wpg;
                bb = bpw;
            }
        }
    // AEQ schedule (waves per half for the long chains and for the rest, and
    // where the longest-first table splits), on scratch copies of the tap state
    const size_t nch = p->aeq_host.size();
    int16_t *tscratch = nullptr;
    AeqItem *tdev = nullptr;
    double best_aeq = 1e30;
    int bq = p->wpp, bql = p->wpp_long;
    size_t bnl = p->n_long, bnd = 0, btop = 0, bfp = 0;
    int blf = -1, btf = -1, bfl = 0;
    bool bfs = false;
    if (p->variant == 0 && hipMalloc(&tscratch, nch * 256 * sizeof(int16_t)) == hipSuccess &&
        hipMalloc(&tdev, nch * sizeof(AeqItem)) == hipSuccess) {
        std::vector<AeqItem> tab = p->aeq_host;
        hipError_t e = hipSuccess;
        for (size_t i = 0; i < nch && e == hipSuccess; ++i) {
            e = hipMemcpyAsync(tscratch + i * 256, tab[i].taps, 256 * sizeof(int16_t),
                               hipMemcpyDeviceToDevice, s);
            tab[i].taps = tscratch + i * 256;
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(tdev, tab.data(), nch * sizeof(AeqItem), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess) {
            std::vector<size_t> splits = {0};
            const uint64_t longest = (p->aeq_host[0].m + 15) / 16;
            // split points: channels whose chain is at least 2/3, 1/2, 1/3, ... 1/64 of the longest
            const int ratio[][2] = {{2, 3}, {1, 2}, {1, 3}, {1, 4}, {1, 6}, {1, 8}, {1, 12}, {1, 16}, {1, 32}, {1, 64}};
            for (const auto &r : ratio) {
                size_t k = 0;
                while (k < nch && (p->aeq_host[k].m + 15) / 16 * (uint64_t)r[1] >= longest * (uint64_t)r[0]) ++k;
                if (k > 0 && k < nch) splits.push_back(k);
            }
            // and fixed counts of longest chains
            for (size_t k = 16; k < nch && k <= 2048; k *= 2) splits.push_back(k);
            std::sort(splits.begin(), splits.end());
            splits.erase(std::unique(splits.begin(), splits.end()), splits.end());
            AeqItem *saved = p->aeq_dev;
            p->aeq_dev = tdev;
            struct Cand { size_t nl; int ql, q; double ms; };
            std::vector<Cand> cands;
            auto time_aeq = [&](const Cand &c) {
                p->n_long = c.nl;
                p->wpp_long = c.ql;
                p->wpp = c.q;
                return time_it([&] {
                    int rc = plan_launch_aeq(p, s, p->side);
                    return rc ? hipErrorUnknown : hipSuccess;
                });
            };
            reps = 1;                                           // one pass, then the best few again
            if (quick) splits = {nch / 2};                      // quick: half the channels long, one pairing
            for (size_t nl : splits)
                for (int ql : {3, 1, 2, 4})                     // long chains: latency-leaning forms
                for (int q : {0, 3, 1, 2, 4}) {
                    if (quick && !(ql == 1 && q == 3)) continue;
                    if (nl == 0 && ql != 4) continue;           // no split: one form for all
                    if (nl > 0 && form_rank(q) >= form_rank(ql)) continue;  // cheaper form for the rest
                    Cand c{nl, ql, q, 0};
                    c.ms = time_aeq(c);
                    cands.push_back(c);
                }
            // the best few again (run-to-run spread is several percent)
            std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.ms < b.ms; });
            for (size_t i = 0; i < cands.size() && i < 4; ++i)
                for (int rep = 0; rep < 2; ++rep) cands[i].ms = std::min(cands[i].ms, time_aeq(cands[i]));
            for (size_t i = 0; i < cands.size() && i < 4; ++i)
                if (cands[i].ms < best_aeq) {
                    best_aeq = cands[i].ms;
                    bq = cands[i].q;
                    bql = cands[i].ql;
                    bnl = cands[i].nl;
                }
            // pipelined lead (whole runs, CDC + AEQ, timed): the lead's size and
            // form, how many of the following chains still take a latency form
            // (the long chains' form chosen above, or two lanes per transform),
            // and the form of the rest
            p->wpg = bw;
            p->bpw = bb;
            struct LCand { size_t lead, nl; int q, ql, lf; size_t top; int tf; double ms; };
            std::vector<LCand> leads;
            auto time_lead = [&](const LCand &c) -> double {
                p->n_lead = c.lead;
                p->n_top = c.top;
                p->n_long = c.nl;
                p->wpp = c.q;
                p->wpp_long = c.ql;
                p->lead_form = c.lf;
                p->top_form = c.tf;
                if (plan_build_segments(p, plan_cdc_top(p), c.lead, s)) return 1e30;
                if (plan_lead(p) != c.lead || plan_top(p) != c.top) return 1e30;
                return time_it([&] { return plan_launch(p, s, p->side, p->side2) ? hipErrorUnknown : hipSuccess; });
            };
            // one pass over all, then the best six by the median of five more;
            // FNT_TUNE_LOG names a file that receives every timing (diagnostics)
            const char *log_path = std::getenv("FNT_TUNE_LOG");
            std::ofstream tlog;
            if (log_path) tlog.open(log_path, std::ios::app);
            auto log_c = [&](const char *what, const LCand &c) {
                if (tlog.is_open())
                    tlog << what << " lead " << c.lead << " long " << c.nl << " q " << c.q << " ql " << c.ql << " lf "
                         << c.lf << " top " << c.top << " tf " << c.tf << " wpg " << p->wpg << " ms " << c.ms << "\n";
            };
            auto best_of = [&](std::vector<LCand> &cs) {
                for (LCand &c : cs) {
                    c.ms = time_lead(c);
                    log_c("pass", c);
                }
                std::sort(cs.begin(), cs.end(), [](const LCand &x, const LCand &y) { return x.ms < y.ms; });
                for (size_t i = 0; i < cs.size() && i < 6; ++i) {
                    double r[5];
                    for (double &v : r) v = time_lead(cs[i]);
                    std::sort(r, r + 5);
                    cs[i].ms = r[2];
                    log_c("median", cs[i]);
                }
                std::sort(cs.begin(), cs.begin() + std::min<size_t>(6, cs.size()),
                          [](const LCand &x, const LCand &y) { return x.ms < y.ms; });
                return cs.front();
            };
            leads.push_back({0, bnl, bq, bql, -1, 0, -1, 0});   // the choice above, without a lead
            // lead forms: one, two and four waves per half (form 5 pairs the
            // halves in a workgroup); following latency chains: the sweep's
            // choice, two lanes per transform, or the pol forms; the rest: one
            // lane or two lanes per transform, or one wave per half
            std::vector<int> lfs = {1, 5, 2, kFusedLead}, qls = {bql}, qs = {0, 3, 1};
            for (int f : {3, 1, 5})
                if (f != bql) qls.push_back(f);
            for (size_t lead : {256, 512, 1024, 1536, 2048})
                for (size_t extra : {0, 512, 1024, 1536})
                    for (int q : qs)
                        for (int lf : lfs)
                            for (int ql : qls) {
                                const size_t nl = lead + extra;
                                if (lead >= nch || nl > nch) continue;
                                // quick: three leads with the latency form after them
                                if (quick && !(lf == 1 && q == 3 && ql == bql && extra == lead &&
                                               (lead == 512 || lead == 1024 || lead == 2048)))
                                    continue;
                                if (extra == 0 && ql != bql) continue;  // no latency form after the lead
                                if (extra > 0 && form_rank(q) >= form_rank(ql)) continue;
                                leads.push_back({lead, nl, q, ql, lf, 0, -1, 0});
                            }
            // (a first lead level on a stream of its own is not among the
            // candidates: single passes sometimes timed it faster, steady runs
            // slower, 130 against 106 ms on the 4096-channel batch)
            LCand best = best_of(leads);
            // the very longest chains of the lead on two waves per half, first in
            // the lead's own launch (form 2 with the rest of the lead in form 5);
            // tried only when the lead already runs in form 5 (as a lead, form 5
            // timed 124 against 105 ms for form 1 on the 4096-channel batch)
            if (best.lead > 0 && best.lf == 5) {
                std::vector<LCand> tops = {best};
                for (size_t top : {32, 64, 128, 256})
                    if (top < best.lead) {
                        LCand c = best;
                        c.top = top;
                        c.tf = 2;
                        c.lf = 5;
                        tops.push_back(c);
                    }
                if (tops.size() > 1) best = best_of(tops);
            }
            p->info.tune_run_ms = best.ms;
            // the CDC's waves per workgroup were chosen on the CDC alone; with a
            // lead the CDC shares the chip with the lead's AEQ, so the best
            // schedule is timed again with the other lane-CDC groupings
            if (best.lead > 0 && bb == 0) {
                for (int wpg : {1, 2, 4}) {
                    if (wpg == bw) continue;
                    const int keep = p->wpg;
                    p->wpg = wpg;
                    double r[3];
                    for (double &v : r) v = time_lead(best);
                    std::sort(r, r + 3);
                    LCand c = best;
                    c.ms = r[1];
                    log_c("cdc-grouping", c);
                    if (r[1] < p->info.tune_run_ms) {
                        p->info.tune_run_ms = r[1];
                        bw = wpg;
                    } else {
                        p->wpg = keep;
                    }
                }
                p->wpg = bw;
            }
            bnd = best.lead;
            bnl = best.nl;
            bq = best.q;
            bql = best.ql;
            blf = best.lf;
            btop = best.top;
            btf = best.tf;
            // the fused persistent kernel (one launch, the 1-sps stream kept in LDS):
            // one wave per half for any batch; two or four waves per half only when
            // every channel is resident at once; channels at raised priority from
            // none to the first 2048.  One pass, then the median of three for the
            // best two, against the staged or lead schedule's median
            {
                struct FCand { int lpt; bool split; size_t prio; double ms; };
                std::vector<FCand> fc;
                for (int lpt : {4, 8, 16}) {
                    const int cap = fused_capacity(lpt);
                    if (cap <= 0 || (quick && lpt != 4)) continue;
                    if (lpt == 4 || nch <= (size_t)cap)
                        for (size_t prio : {0, 256, 512, 1024, 2048})
                            if ((prio == 0 || prio < nch) && (!quick || prio == 0 || prio == 512))
                                fc.push_back({lpt, false, prio, 0});
                    // a workgroup per half when the halves of every channel fit at once
                    if (2 * nch <= (size_t)cap && !quick) fc.push_back({lpt, true, nch, 0});
                }
                auto time_fused = [&](const FCand &c) {
                    p->fused_lpt = c.lpt;
                    p->fused_split = c.split;
                    p->fused_prio = c.prio;
                    p->fused_grid = plan_fused_grid(p, c.lpt, c.split);
                    double ms = time_it([&] { return plan_launch(p, s, p->side, p->side2) ? hipErrorUnknown : hipSuccess; });
                    if (tlog.is_open())
                        tlog << "fused lpt " << c.lpt << " split " << c.split << " prio " << c.prio << " grid "
                             << p->fused_grid << " ms " << ms << "\n";
                    return ms;
                };
                for (FCand &c : fc) c.ms = time_fused(c);
                std::sort(fc.begin(), fc.end(), [](const FCand &x, const FCand &y) { return x.ms < y.ms; });
                FCand fbest{0, false, 0, 1e30};
                for (size_t i = 0; i < fc.size() && i < 2; ++i) {
                    double r[3];
                    for (double &v : r) v = time_fused(fc[i]);
                    std::sort(r, r + 3);
                    if (r[1] < fbest.ms) fbest = {fc[i].lpt, fc[i].split, fc[i].prio, r[1]};
                }
                p->fused_lpt = 0;
                p->fused_split = false;
                if (fbest.lpt && fbest.ms < p->info.tune_run_ms) {
                    bfl = fbest.lpt;
                    bfs = fbest.split;
                    bfp = fbest.prio;
                    p->info.tune_run_ms = fbest.ms;
                }
            }
            p->n_lead = p->n_top = 0;
            p->lead_form = p->top_form = -1;
            p->seg_lead = p->seg_top = 0;
            p->aeq_dev = saved;
        }
    }
    if (tscratch) (void)hipFree(tscratch);
    if (tdev) (void)hipFree(tdev);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->wpg = bw;
    p->bpw = bb;
    p->wpp = bq;
    p->wpp_long = bql;
    p->n_long = bnl;
    p->n_lead = bnd;
    p->lead_form = blf;
    p->n_top = btop;
    p->top_form = btf;
    p->fused_lpt = bfl;
    p->fused_split = bfs;
    p->fused_prio = bfp;
    if (bfl) p->fused_grid = plan_fused_grid(p, bfl, p->fused_split);
    p->info.tune_ms = best_aeq < 1e29 ? best_aeq : best_cdc;
    // the cache keeps a split fused schedule as a negative lane count
    tune_cache_store(cache, key, bw, bb, bq, bql, (long long)bnl, (long long)bnd, blf, (long long)btop, btf,
                     bfs ? -bfl : bfl, (long long)bfp, p->info.tune_ms);
    return FNT_OK;
}

extern "C" {

int fnt_plan_create(fnt_plan **out, const fnt_channel_desc *ch, size_t nch, const fnt_plan_config *cfg,
                    void *stream) {
    if (!out) return fail(FNT_E_INVAL, "plan: NULL out");
    *out = nullptr;
    if (nch > 0 && !ch) return fail(FNT_E_INVAL, "plan: NULL channel table");
    if (nch > (size_t)0x7FFFFFFF) return fail(FNT_E_INVAL, "plan: too many channels");
    fnt_plan_config c{};
    if (cfg) c = *cfg;
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (cfg && c.device != dev) {
        hipError_t e = hipSetDevice(c.device);
        if (e != hipSuccess) return hip_fail(e, "plan: hipSetDevice");
        dev = c.device;
    }
    hipStream_t s = (hipStream_t)stream;
    fnt_plan *p = new fnt_plan();
    p->device = dev;
    int rc = device_err_flag(&p->err);
    if (rc) {
        delete p;
        return rc;
    }
    uint64_t sym_total = 0, blocks = 0, chunks = 0, inst = 0, chain_max = 0;
    std::vector<uint64_t> aoff(nch);
    for (size_t i = 0; i < nch; ++i) {
        const fnt_channel_desc &d = ch[i];
        if ((rc = validate_cdc(&d.cdc)) || (rc = validate_aeq(&d.aeq))) {
            delete p;
            return fail(rc, "plan: channel %zu: %s", i, fnt_last_error());
        }
        if (!d.taps || (d.n > 0 && !d.in) || (n_symbols(d.n, d.cdc.decim_phase) > 0 && !d.out) ||
            !aligned(d.in, 4) || !aligned(d.out, 8) ||
            !aligned(d.taps, 2)) {
            delete p;
            return fail(FNT_E_INVAL, "plan: channel %zu: NULL or misaligned buffer", i);
        }
        uint64_t M = n_symbols(d.n, d.cdc.decim_phase);
        aoff[i] = sym_total;
        sym_total += (M + 3) & ~3ull;   // keep each channel's scratch 16-byte aligned
        inst += d.n;
        chain_max = std::max(chain_max, (M + 15) / 16);
    }
    if (sym_total > 0) {
        hipError_t e = hipMalloc(&p->abuf, sym_total * 4);
        if (e != hipSuccess) {
            delete p;
            (void)hipGetLastError();   // not left for the caller's next launch check
            return fail(FNT_E_NOMEM, "plan: scratch of %llu bytes: %s", (unsigned long long)(sym_total * 4),
                        hipGetErrorString(e));
        }
    }
    // both tables longest AEQ chain first (the chains bound the makespan), in
    // the same order, so that a prefix of channels is a prefix of each table
    std::vector<size_t> order(nch);
    for (size_t i = 0; i < nch; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        return n_symbols(ch[a].n, ch[a].cdc.decim_phase) > n_symbols(ch[b].n, ch[b].cdc.decim_phase);
    });
    p->cdc_host.resize(nch);
    p->aeq_host.resize(nch);
    for (size_t k = 0; k < nch; ++k) {
        const size_t i = order[k];
        const fnt_channel_desc &d = ch[i];
        CdcItem &ci = p->cdc_host[k];
        fill_cdc_item(ci, d.in, d.n, &d.cdc);
        ci.a_out = p->abuf + aoff[i] * 4;
        ci.block0 = blocks;
        ci.chunk0 = chunks;
        blocks += cdc_blocks(d.n);
        chunks += cdc_chunks(d.n);
        AeqItem &ai = p->aeq_host[k];
        fill_aeq_item(ai, ci.a_out, n_symbols(d.n, d.cdc.decim_phase), d.taps, &d.aeq, d.out);
    }
    p->total_blocks = blocks;
    p->total_chunks = chunks;
    hipError_t e = hipSuccess;
    if (nch > 0) {
        e = hipMalloc(&p->cdc_dev, nch * sizeof(CdcItem));
        if (e == hipSuccess) e = hipMalloc(&p->aeq_dev, nch * sizeof(AeqItem));
        if (e != hipSuccess) {
            fnt_plan_destroy(p);
            (void)hipGetLastError();   // not left for the caller's next launch check
            return fail(FNT_E_NOMEM, "plan: tables: %s", hipGetErrorString(e));
        }
        e = hipMemcpyAsync(p->cdc_dev, p->cdc_host.data(), nch * sizeof(CdcItem), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(p->aeq_dev, p->aeq_host.data(), nch * sizeof(AeqItem), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            fnt_plan_destroy(p);
            return hip_fail(e, "plan: upload tables");
        }
    }
    if (nch > 0) {
        hipError_t eq = hipMalloc(&p->queue, 2 * sizeof(uint32_t));
        if (eq != hipSuccess) {
            fnt_plan_destroy(p);
            (void)hipGetLastError();   // not left for the caller's next launch check
            return fail(FNT_E_NOMEM, "plan: work counter: %s", hipGetErrorString(eq));
        }
        eq = hipMemset(p->queue, 0, 2 * sizeof(uint32_t));
        if (eq != hipSuccess) {
            fnt_plan_destroy(p);
            return hip_fail(eq, "plan: clear work counter");
        }
    }
    default_cdc_schedule(blocks, &p->wpg, &p->bpw);
    p->wpp = default_wpp(nch);
    p->wpp_long = 4;
    p->n_long = 0;
    {
        hipError_t ee = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
        if (ee == hipSuccess) ee = hipStreamCreateWithFlags(&p->side2, hipStreamNonBlocking);
        if (ee == hipSuccess) ee = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
        if (ee == hipSuccess) ee = hipEventCreateWithFlags(&p->join, hipEventDisableTiming);
        if (ee == hipSuccess) ee = hipEventCreateWithFlags(&p->fork2, hipEventDisableTiming);
        if (ee == hipSuccess) ee = hipEventCreateWithFlags(&p->join2, hipEventDisableTiming);
        if (ee != hipSuccess) {
            fnt_plan_destroy(p);
            return hip_fail(ee, "plan: side stream");
        }
    }
    if (c.autotune && blocks > 0) {
        if ((rc = plan_autotune(p, s, c.tune_cache, c.tune_quick != 0))) {
            fnt_plan_destroy(p);
            return rc;
        }
    }
    if ((rc = plan_build_segments(p, plan_cdc_top(p), p->n_lead, s))) {
        fnt_plan_destroy(p);
        return rc;
    }
    p->use_graph = c.use_graph != 0;
    if (p->use_graph && nch > 0) {
        if ((rc = plan_capture(p, s))) {
            fnt_plan_destroy(p);
            return rc;
        }
    }
    p->info.channels = nch;
    p->info.instants = inst;
    p->info.symbols = 0;
    for (auto &a : p->aeq_host) p->info.symbols += a.m;
    p->info.cdc_blocks = blocks;
    p->info.aeq_blocks_max = chain_max;
    *out = p;
    return FNT_OK;
}

int fnt_plan_run(fnt_plan *p, void *stream) {
    if (!p) return fail(FNT_E_INVAL, "plan: NULL");
    if (p->cdc_host.empty()) return FNT_OK;
    hipStream_t s = (hipStream_t)stream;
    if (p->exec) {                                    // a lead's branch is forked and joined inside the graph
        hipError_t e = hipGraphLaunch(p->exec, s);
        if (e != hipSuccess) return hip_fail(e, "plan: graph launch");
        return FNT_OK;
    }
    return plan_launch(p, s, p->side, p->side2);
}

int fnt_plan_run_graph(fnt_plan *p, void *stream) {
    if (!p) return fail(FNT_E_INVAL, "plan: NULL");
    if (p->cdc_host.empty()) return FNT_OK;
    if (!p->exec) return fail(FNT_E_STATE, "plan: no captured graph (created without use_graph)");
    hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "plan: graph launch");
    return FNT_OK;
}

int fnt_plan_run_stage(fnt_plan *p, int stages, void *stream) {
    if (!p) return fail(FNT_E_INVAL, "plan: NULL");
    if (stages & ~FNT_STAGE_ALL) return fail(FNT_E_INVAL, "plan: stage mask 0x%x", stages);
    if (p->cdc_host.empty()) return FNT_OK;
    hipStream_t s = (hipStream_t)stream;
    int rc = FNT_OK;
    if (stages & FNT_STAGE_CDC) rc = plan_launch_cdc(p, s);
    if (!rc && (stages & FNT_STAGE_AEQ)) rc = plan_launch_aeq(p, s, p->side);
    return rc;
}

int fnt_plan_get_info(const fnt_plan *p, fnt_plan_info *info) {
    if (!p || !info) return fail(FNT_E_INVAL, "plan info: NULL");
    *info = p->info;
    info->cdc_waves_per_group = p->wpg;
    info->cdc_blocks_per_wave = p->bpw;
    info->aeq_variant = p->variant;
    info->aeq_waves_per_pol = p->wpp;
    info->aeq_waves_long = p->wpp_long;
    info->aeq_long_channels = p->variant == 0 ? std::min(p->n_long, p->aeq_host.size()) : 0;
    info->graph = p->exec ? 1 : 0;
    info->cdc_variant = p->cdc_variant;
    const size_t lead = plan_lead(p);
    info->lead_channels = (int32_t)lead;
    info->lead_form = p->lead_form >= 0 ? p->lead_form : p->wpp_long;
    info->top_channels = lead ? (int32_t)plan_top(p) : 0;
    info->top_form = p->top_form >= 0 ? p->top_form : p->wpp_long;
    info->fused_lpt = p->fused_lpt;
    info->fused_grid = p->fused_lpt ? (int32_t)p->fused_grid : 0;
    info->fused_prio_channels = p->fused_lpt ? std::min(p->fused_prio, p->aeq_host.size()) : 0;
    info->fused_split = p->fused_lpt && p->fused_split ? 1 : 0;
    return FNT_OK;
}

int fnt_plan_set_fused(fnt_plan *p, int lpt, uint64_t prio_channels, int split_halves) {
    if (!p) return fail(FNT_E_INVAL, "plan: NULL");
    if (lpt != 0 && lpt != 4 && lpt != 8 && lpt != 16)
        return fail(FNT_E_INVAL, "plan: fused lanes per transform %d (0, 4, 8 or 16)", lpt);
    if (split_halves != 0 && split_halves != 1) return fail(FNT_E_INVAL, "plan: split_halves %d", split_halves);
    p->fused_lpt = lpt;
    p->fused_split = split_halves != 0;
    p->fused_prio = (size_t)std::min<uint64_t>(prio_channels, p->aeq_host.size());
    p->fused_grid = lpt ? plan_fused_grid(p, lpt, p->fused_split) : 0;
    if (p->exec) return plan_capture(p, nullptr);
    return FNT_OK;
}

int fnt_plan_set_lead(fnt_plan *p, uint64_t lead, int lead_form, uint64_t top, int top_form) {
    if (!p) return fail(FNT_E_INVAL, "plan: NULL");
    p->fused_lpt = 0;                                // another schedule: the fused kernel is off
    if (lead_form != -1 && lead_form != kFusedLead && !valid_form(lead_form))
        return fail(FNT_E_INVAL, "plan: lead form %d", lead_form);
    if (top_form != -1 && !valid_form(top_form)) return fail(FNT_E_INVAL, "plan: first-level form %d", top_form);
    const size_t n = p->aeq_host.size();
    const size_t l = lead < n ? (size_t)lead : 0;
    const size_t t = top < l ? (size_t)top : 0;
    // the segmented table may be read by runs still in flight on any stream
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "plan: set lead");
    p->n_lead = l;
    p->n_top = t;
    p->lead_form = lead_form;
    p->top_form = top_form;
    int rc = plan_build_segments(p, plan_cdc_top(p), l, nullptr);
    if (rc) return rc;
    if (p->exec) return plan_capture(p, nullptr);
    return FNT_OK;
}

int fnt_plan_run_timed(fnt_plan *p, fnt_plan_timing *t, void *stream) {
    if (!p || !t) return fail(FNT_E_INVAL, "plan run timed: NULL");
    std::memset(t, 0, sizeof *t);
    if (p->cdc_host.empty()) return FNT_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    for (int i = 0; i < 8 && e == hipSuccess; ++i)
        if (!p->tev[i]) e = hipEventCreate(&p->tev[i]);
    if (e != hipSuccess) return hip_fail(e, "plan: timing events");
    const size_t lead = plan_lead(p);
    const size_t top = lead && !plan_top_fused(p) ? plan_top(p) : 0;   // a launch of its own
    int rc = plan_launch(p, s, p->side, p->side2, p->tev);
    if (rc) return rc;
    e = hipEventSynchronize(p->tev[5]);
    float ms = 0;
    auto el = [&](int a, int b, float *out) {
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p->tev[a], p->tev[b]);
        if (e == hipSuccess) *out = ms;
    };
    el(0, 5, &t->step_ms);
    el(0, 1, &t->cdc_ms);
    el(1, 4, &t->aeq_ms);
    if (lead) el(2, 3, &t->aeq_lead_ms);
    if (top) el(6, 7, &t->aeq_top_ms);
    if (e != hipSuccess) return hip_fail(e, "plan: timing");
    t->aeq_top_blocks = aeq_blocks_of(p, 0, top);
    t->aeq_lead_blocks = aeq_blocks_of(p, top, lead);
    t->aeq_blocks = aeq_blocks_of(p, lead, p->aeq_host.size());
    t->fused = p->fused_lpt ? 1 : 0;
    return FNT_OK;
}

int fnt_plan_set_aeq_variant(fnt_plan *p, int variant) {
    if (!p) return fail(FNT_E_INVAL, "plan: NULL");
    p->fused_lpt = 0;                                // another schedule: the fused kernel is off
    if (variant < 0 || variant > 3) return fail(FNT_E_INVAL, "plan: variant %d", variant);
    p->variant = variant;
    if (p->exec) return plan_capture(p, nullptr);
    return FNT_OK;
}

int fnt_plan_set_cdc_variant(fnt_plan *p, int variant) {
    if (!p) return fail(FNT_E_INVAL, "plan: NULL");
    p->fused_lpt = 0;                                // another schedule: the fused kernel is off
    if (variant != 0 && variant != 1) return fail(FNT_E_INVAL, "plan: CDC variant %d", variant);
    p->cdc_variant = variant;
    if (p->exec) return plan_capture(p, nullptr);
    return FNT_OK;
}

int fnt_plan_set_aeq_waves(fnt_plan *p, int wpp) {
    if (!p) return fail(FNT_E_INVAL, "plan: NULL");
    p->fused_lpt = 0;                                // another schedule: the fused kernel is off
    if (!valid_form(wpp)) return fail(FNT_E_INVAL, "plan: AEQ form %d", wpp);
    p->wpp = wpp;
    p->n_long = 0;
    p->n_lead = p->n_top = 0;
    if (p->exec) return plan_capture(p, nullptr);
    return FNT_OK;
}

int fnt_plan_set_aeq_split(fnt_plan *p, uint64_t long_channels, int wpp_long, int wpp) {
    if (!p) return fail(FNT_E_INVAL, "plan: NULL");
    p->fused_lpt = 0;                                // another schedule: the fused kernel is off
    if (!valid_form(wpp_long) || !valid_form(wpp))
        return fail(FNT_E_INVAL, "plan: waves per half %d / %d", wpp_long, wpp);
    p->n_long = (size_t)std::min<uint64_t>(long_channels, p->aeq_host.size());
    p->wpp_long = wpp_long;
    p->wpp = wpp;
    if (p->exec) return plan_capture(p, nullptr);
    return FNT_OK;
}

int fnt_plan_set_cdc_schedule(fnt_plan *p, int wpg, int bpw) {
    if (!p) return fail(FNT_E_INVAL, "plan: NULL");
    if (wpg != 1 && wpg != 2 && wpg != 4) return fail(FNT_E_INVAL, "plan: waves per group %d", wpg);
    if (bpw < 0 || bpw > 1024) return fail(FNT_E_INVAL, "plan: blocks per wave %d", bpw);
    p->wpg = wpg;
    p->bpw = bpw;
    if (p->exec) return plan_capture(p, nullptr);
    return FNT_OK;
}

int fnt_plan_destroy(fnt_plan *p) {
    if (!p) return FNT_OK;
    plan_drop_graph(p);
    if (p->side) (void)hipStreamDestroy(p->side);
    if (p->side2) (void)hipStreamDestroy(p->side2);
    for (hipEvent_t ev : {p->fork, p->join, p->fork2, p->join2})
        if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : p->tev)
        if (ev) (void)hipEventDestroy(ev);
    if (p->cdc_seg_dev) (void)hipFree(p->cdc_seg_dev);
    if (p->cdc_dev) (void)hipFree(p->cdc_dev);
    if (p->aeq_dev) (void)hipFree(p->aeq_dev);
    if (p->abuf) (void)hipFree(p->abuf);
    if (p->queue) (void)hipFree(p->queue);
    delete p;
    return FNT_OK;
}

}  // extern "C"
