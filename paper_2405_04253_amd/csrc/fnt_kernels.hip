// gfx950 kernels of the FNT-CDC + FNT-AEQ receiver path.
//
//  * fnt_transform_kernel : batched Eq. (1) / Eq. (2) transforms modulo F_2, F_3,
//    F_4 at the full radix order (Fig. 1 case, the AEQ's N = 32 / alpha = 2, the
//    CDC's N = 64 / alpha = sqrt 2, and the F_2 / F_3 variants).
//  * cdc_lane_kernel      : overlap-save FNT-CDC (Fig. 2), one 32-instant block per
//    lane; complex product through the two real Fermat-domain products of
//    Eqs. (7)-(8), exact centred lift of the kept instants, resampling to 1
//    sample/symbol and requantisation to 5 bit.
//  * cdc_kernel           : the same CDC with one block per wave (16 lanes per
//    64-point transform); the only form that also writes the exact output z.
//  * aeq_lane_kernel, aeq_duo_kernel, aeq_pol_kernel<LPT>, aeq_split_kernel:
//    FNT-AEQ (Fig. 3): 4x4 real MIMO filtering in the Fermat domain with 14-bit
//    taps split into two 7-bit digit groups, the RDE error of Eq. (6) and the
//    block tap update, in forms from throughput (one transform per lane) to
//    latency (a channel's polarisation halves over several waves), and a split
//    launch of two forms.
//  * cdc_aeq_fused_kernel : the whole chain (CDC, resampling, AEQ) in one
//    persistent launch: per channel a producer wave runs the lane-per-block CDC
//    64 blocks at a time into a ring in LDS and the polarisation-split AEQ waves
//    consume it; workgroups take channels longest first from a work counter.
//  * aeq_fnt_kernel       : the same AEQ with one wave64 per channel, with the RDE
//    gradient of the tap update as dot products or in the Fermat domain.
//  * cdc_direct_kernel, aeq_direct_kernel : the same CDC and AEQ by time-domain
//    integer dot products, comparators with bit-identical output.
#include <hip/hip_runtime.h>

#include <utility>

#include "fnt_device.hpp"
#include "fnt_internal.hpp"

using namespace fntd;
using fnti::AeqItem;
using fnti::CdcItem;

// Test-only counting build (FNT_COUNT_PRODUCTS=1, a separate library): every
// lane adds the Fermat-domain spectral products it computes (the true
// multiplications Tab. 1 counts) to g_fnt_products[0] (CDC) and [1] (AEQ).
#ifndef FNT_COUNT_PRODUCTS
#define FNT_COUNT_PRODUCTS 0
#endif
#if FNT_COUNT_PRODUCTS
__device__ unsigned long long g_fnt_products[2];
#endif

namespace {

__device__ __forceinline__ void count_products(int which, uint32_t n) {
#if FNT_COUNT_PRODUCTS
    atomicAdd(&g_fnt_products[which], (unsigned long long)n);
#else
    (void)which;
    (void)n;
#endif
}

__device__ __forceinline__ void flag(int *err, int bit) {
    if (err) atomicOr(err, bit);
}

// s_mu of stream block j under the item's step schedule: mu_shift before block
// gear_blocks, mu_shift_late from then on (gear_blocks = 0: mu_shift throughout).
__device__ __forceinline__ int step_shift(const AeqItem &it, uint64_t j) {
    return (it.gear_blocks != 0u && j >= (uint64_t)it.gear_blocks) ? it.mu_shift_late : it.mu_shift;
}

// ---------------------------------------------------------------- transforms --

// Powers of the CDC radix alpha = sqrt 2 = 4080 modulo 65537, alpha^e for e < 64.
struct AlphaPow {
    int32_t v[64];
};
constexpr AlphaPow make_alpha_pow() {
    AlphaPow a{};
    uint64_t x = 1;
    for (int e = 0; e < 64; ++e) {
        a.v[e] = (int32_t)x;
        x = x * 4080u % 65537u;
    }
    return a;
}
__constant__ AlphaPow kAlphaPow = make_alpha_pow();

constexpr uint32_t pow_mod(uint32_t b, uint32_t e, uint32_t m) {
    uint64_t r = 1, x = b % m;
    while (e) {
        if (e & 1) r = r * x % m;
        x = x * x % m;
        e >>= 1;
    }
    return (uint32_t)r;
}

// Transforms across N = 2^LOGN lanes of a wave, one element per lane (position
// pos = lane mod N).  Forward: decimation in frequency, natural order in, lane
// pos ends with X[bitrev(pos)].  Inverse: decimation in time, bit-reversed
// order in, lane pos ends with N x[pos] (unnormalised).  Each radix-2 stage
// exchanges with lane ^ H by a DPP or swizzle move where one exists; residues
// stay canonical in [0, F).
template <int Q, int LOGN, bool SQRT2, int H>
__device__ __forceinline__ uint32_t fwd_stage_x(uint32_t x, int pos) {
    using FF = Field<Q>;
    constexpr int N = 1 << LOGN;
    const uint32_t p = (uint32_t)xor_lane<H>((int32_t)x);
    const int e = (N / (2 * H)) * (pos & (H - 1));
    const uint32_t s = FF::add(x, p);
    const uint32_t d = FF::template mul_radix_pow<SQRT2>(FF::sub(p, x), e);
    return (pos & H) ? d : s;
}
template <int Q, int LOGN, bool SQRT2, int H>
__device__ __forceinline__ uint32_t inv_stage_x(uint32_t x, int pos) {
    using FF = Field<Q>;
    constexpr int N = 1 << LOGN;
    const bool upper = (pos & H) != 0;
    const int e = (N / (2 * H)) * (pos & (H - 1));
    const uint32_t t = upper ? FF::template mul_radix_pow<SQRT2>(x, e ? N - e : 0) : x;
    const uint32_t p = (uint32_t)xor_lane<H>((int32_t)t);
    return upper ? FF::sub(p, t) : FF::add(x, p);
}
template <int Q, int LOGN, bool SQRT2, int H = (1 << LOGN) / 2>
__device__ __forceinline__ uint32_t fwd_dpp(uint32_t x, int pos) {      // stages H = N/2 .. 1
    x = fwd_stage_x<Q, LOGN, SQRT2, H>(x, pos);
    if constexpr (H > 1) return fwd_dpp<Q, LOGN, SQRT2, H / 2>(x, pos);
    else return x;
}
template <int Q, int LOGN, bool SQRT2, int H = 1>
__device__ __forceinline__ uint32_t inv_dpp(uint32_t x, int pos) {      // stages H = 1 .. N/2
    x = inv_stage_x<Q, LOGN, SQRT2, H>(x, pos);
    if constexpr (2 * H < (1 << LOGN)) return inv_dpp<Q, LOGN, SQRT2, 2 * H>(x, pos);
    else return x;
}

// The same transforms modulo 65537 on loose residues (signed int32, reduced
// only inside mulmod): a stage is two DPP-fed sums and one 24-bit product.
// Canonical input (< 2^17); after stage k the sums are below 2^(17+k) and the
// products below 2^17 (the inverse multiplies every value, by 1 in the lower
// lanes, so its sums stay below 2^18), and every mulmod input stays below 2^23
// for N <= 64.
// Twiddles alpha^(+-e), e < 32: 2^e / -2^(16-e) for alpha = 2, the table of
// 4080^e for alpha = sqrt 2.
template <int LOGN, bool SQRT2, int H>
__device__ __forceinline__ int32_t fwd_stage_lazy(int32_t x, int pos) {
    constexpr int N = 1 << LOGN;
    const int e = (N / (2 * H)) * (pos & (H - 1));
    const int32_t c = SQRT2 ? kAlphaPow.v[e] : (1 << e);
    const int32_t p = xor_lane<H>(x);
    const int32_t s = x + p;
    const int32_t d = mulmod(p - x, c);
    return (pos & H) ? d : s;
}
template <int LOGN, bool SQRT2, int H>
__device__ __forceinline__ int32_t inv_stage_lazy(int32_t x, int pos) {
    constexpr int N = 1 << LOGN;
    const bool upper = (pos & H) != 0;
    const int e = upper ? (N / (2 * H)) * (pos & (H - 1)) : 0;
    // every lane multiplies (lower lanes by 1): no branch, and the twiddle load
    // does not depend on the data, so it leaves the loop
    const int32_t c = SQRT2 ? kAlphaPow.v[(N - e) & (N - 1)] : (e ? -(1 << (16 - e)) : 1);
    const int32_t t = mulmod(x, c);
    const int32_t p = xor_lane<H>(t);
    return upper ? p - t : t + p;
}
template <int LOGN, bool SQRT2, int H = (1 << LOGN) / 2>
__device__ __forceinline__ int32_t fwd_lazy(int32_t x, int pos) {
    x = fwd_stage_lazy<LOGN, SQRT2, H>(x, pos);
    if constexpr (H > 1) return fwd_lazy<LOGN, SQRT2, H / 2>(x, pos);
    else return x;
}
template <int LOGN, bool SQRT2, int H = 1>
__device__ __forceinline__ int32_t inv_lazy(int32_t x, int pos) {
    x = inv_stage_lazy<LOGN, SQRT2, H>(x, pos);
    if constexpr (2 * H < (1 << LOGN)) return inv_lazy<LOGN, SQRT2, 2 * H>(x, pos);
    else return x;
}
// A loose residue mod 65537 (|v| < 2^31) to canonical [0, 65537).
__device__ __forceinline__ uint32_t canon65537(int32_t v) {
    int32_t f = (int32_t)((uint32_t)v & 0xFFFFu) - (v >> 16);      // (-2^15, 2^16 + 2^15)
    f = f < 0 ? f + 65537 : f;
    return (uint32_t)(f >= 65537 ? f - 65537 : f);
}

// Grid-stride over the batch: the stride is a multiple of 64, so a lane keeps
// its position and its twiddles, and the lanes of one vector enter and leave
// the loop together (their exchanges never read a lane that has left).
template <int Q, int LOGN, bool SQRT2, bool INV>
__global__ __launch_bounds__(256) void fnt_transform_kernel(const uint32_t *x, uint32_t *X,
                                                            uint64_t total, int *err) {
    using FF = Field<Q>;
    constexpr int N = 1 << LOGN;
    constexpr uint32_t NINV = pow_mod(N, FF::F - 2, FF::F);
    const int pos = (int)(threadIdx.x & 63) & (N - 1);
    const int rpos = bitrev(pos, LOGN);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; gid - (uint64_t)pos < total;
         gid += stride) {
        const uint64_t base = gid - (uint64_t)pos;
        uint32_t v = x[INV ? base + (uint64_t)rpos : gid];
        if (v >= FF::F) {
            bad = true;
            v %= FF::F;
        }
        if constexpr (Q == 16) {
            constexpr int32_t NINV_S = NINV > FF::F / 2 ? (int32_t)NINV - (int32_t)FF::F : (int32_t)NINV;
            if constexpr (!INV)
                v = canon65537(fwd_lazy<LOGN, SQRT2>((int32_t)v, pos));
            else
                v = canon65537(mulmod(inv_lazy<LOGN, SQRT2>((int32_t)v, pos), NINV_S));
        } else if constexpr (!INV) {
            v = fwd_dpp<Q, LOGN, SQRT2>(v, pos);
        } else {
            v = FF::mul(inv_dpp<Q, LOGN, SQRT2>(v, pos), NINV);
        }
        X[INV ? gid : base + (uint64_t)rpos] = v;
    }
    if (bad) flag(err, RANGE_RESIDUE);
}

// ----------------------------------------------------------------------- CDC --

// LDS hand-off between lanes of one wave: LDS instructions of a wave are
// processed in issue order, so only the compiler must not move memory
// operations across this point.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The polarisation-split AEQ: words per stream row of its input spectra (rows
// 16-byte aligned for the batched stores); blocks per batch and bytes per
// stream row of a batch's staged window symbols (144 used, the tail zero).
constexpr int kSpecRow = 36;
constexpr int kBatch = 8;
constexpr int kStgRow = 160;
typedef int32_t v16i __attribute__((ext_vector_type(16)));

// The 5-bit reversal of p.
__device__ __forceinline__ int bitrev5(int p) {
    return ((p & 1) << 4) | ((p & 2) << 2) | (p & 4) | ((p & 8) >> 2) | ((p & 16) >> 4);
}

// Wait until every vector memory operation of this wave has completed
// (s_waitcnt vmcnt(0); expcnt and lgkmcnt fields left at their maxima), and keep
// the compiler from moving later memory operations above the wait.
__device__ __forceinline__ void vmem_wait_all() {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __builtin_amdgcn_sched_barrier(0);
}


// All bytes of w in [-16, 15]: the top four bits of each byte are equal.
__device__ __forceinline__ bool bytes_5bit(uint32_t w) {
    return ((w ^ (w << 1)) & 0xE0E0E0E0u) == 0u;
}

__device__ __forceinline__ int8_t sbyte(uint32_t w, int k) { return (int8_t)(w >> (8 * k)); }

__device__ __forceinline__ uint32_t cdc_load(const CdcItem &it, int64_t i) {
    if (i < 0) {
        return it.hist ? reinterpret_cast<const uint32_t *>(it.hist)[32 + i] : 0u;
    }
    return (uint64_t)i < it.n ? reinterpret_cast<const uint32_t *>(it.in)[i] : 0u;
}


// 64-point transforms of the CDC, 16 lanes per transform, 4 points per lane:
// lane t of a group holds positions n = t + 16 j (j < 4).  Twiddle constants
// of this lane for the forward (alpha^e) and inverse (alpha^-e) transforms.
struct CdcTw {
    int32_t f32[2], f16, fx[4];    // forward: h = 32 (j = 0, 1), h = 16, h = 8, 4, 2, 1
    int32_t i32[2], i16, ix[4];    // inverse: the same exponents negated
};
__device__ __forceinline__ CdcTw cdc_twiddles(int t) {
    CdcTw w;
    const int32_t *ap = kAlphaPow.v;
    w.f32[0] = ap[t];
    w.f32[1] = ap[t + 16];
    w.f16 = ap[2 * t];
    w.i32[0] = ap[(64 - t) & 63];
    w.i32[1] = ap[(64 - t - 16) & 63];
    w.i16 = ap[(64 - 2 * t) & 63];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int h = 8 >> q;
        const int e = (32 / h) * (t & (h - 1));
        w.fx[q] = ap[e];
        w.ix[q] = ap[(64 - e) & 63];
    }
    return w;
}

// DIF forward, in: |x| < 2^15; out: |X| < 2^22, register j holds bin bitrev6(t + 16 j).
__device__ __forceinline__ void cdc_fnt64(int32_t (&x)[4], int t, const CdcTw &w) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {                       // h = 32
        int32_t a = x[j], b = x[j + 2];
        x[j] = a + b;
        x[j + 2] = mulmod(a - b, w.f32[j]);
    }
#pragma unroll
    for (int j = 0; j < 4; j += 2) {                    // h = 16
        int32_t a = x[j], b = x[j + 1];
        x[j] = a + b;
        x[j + 1] = mulmod(a - b, w.f16);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {                       // h = 8, 4, 2, 1 across lanes
        const int h = 8 >> q;
        const bool up = (t & h) != 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int32_t p = h == 8 ? xor_pos<8>(x[j]) : h == 4 ? xor_pos<4>(x[j])
                      : h == 2 ? xor_pos<2>(x[j]) : xor_pos<1>(x[j]);
            x[j] = blend(up, mulmod(p - x[j], w.fx[q]), x[j] + p);
        }
    }
}

// DIT inverse (unnormalised) keeping positions 32..63 (registers 2, 3).
// In: |x| < 2^18; out: |x| < 2^20.
__device__ __forceinline__ void cdc_ifnt64_upper(int32_t (&x)[4], int t, const CdcTw &w) {
#pragma unroll
    for (int q = 3; q >= 0; --q) {                      // h = 1, 2, 4, 8 across lanes
        const int h = 8 >> q;
        const bool up = (t & h) != 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int32_t tt = blend(up, mulmod(x[j], w.ix[q]), x[j]);
            int32_t p = h == 8 ? xor_pos<8>(tt) : h == 4 ? xor_pos<4>(tt)
                      : h == 2 ? xor_pos<2>(tt) : xor_pos<1>(tt);
            x[j] = blend(up, p - tt, x[j] + p);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; j += 2) {                    // h = 16
        int32_t tt = mulmod(x[j + 1], w.i16);
        int32_t a = x[j];
        x[j] = a + tt;
        x[j + 1] = a - tt;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j)                         // h = 32: upper half only
        x[j + 2] = x[j] - mulmod(x[j + 2], w.i32[j]);
}

// Tap spectra of this lane's group: g = 2 pol + uv, uv = 0: H+ = FNT64(h_r + 2^8 h_i),
// uv = 1: H- = FNT64(h_r - 2^8 h_i) (the per-channel factors of Eqs. (7)-(8)).
__device__ __forceinline__ void cdc_tap_spectra(const int8_t *taps, int ntaps, int uv, int t,
                                                const CdcTw &w, int32_t (&H)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = t + 16 * j;
        int32_t hr = 0, hi = 0;
        if (k < ntaps) {
            hr = taps[2 * k];
            hi = taps[2 * k + 1];
        }
        H[j] = uv ? hr - 256 * hi : hr + 256 * hi;
    }
    cdc_fnt64(H, t, w);
}

// Overlap-save FNT-CDC.  One wave per 32-instant block (contiguous ranges of
// blocks per wave); the 64-instant window is transformed as four 64-point
// sequences u_X, v_X, u_Y, v_Y (u = x_r + 2^8 x_i, v = x_r - 2^8 x_i, Eqs. (7)-(8)
// by linearity), one per 16-lane group.
template <bool WITH_Z>
__global__ __launch_bounds__(256) void cdc_kernel(const CdcItem *items, int nitems,
                                                  CdcItem single, uint64_t total_blocks,
                                                  int blocks_per_wave, int *err) {
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int g = lane >> 4, t = lane_pos(lane & 15);   // t: position index of the lane
    const int pol = g >> 1, uv = g & 1;
    __shared__ uint32_t winw_s[4][64];                 // per wave: the 64-instant window
    __shared__ uint32_t outw_s[4][32];                 // per wave: requantised bytes [instant][comp]
    uint32_t *winw = winw_s[wv];
    uint32_t *outw = outw_s[wv];

    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wv;
    const uint64_t b_begin = wave * (uint64_t)blocks_per_wave;
    if (b_begin >= total_blocks) return;
    uint64_t b_end = b_begin + (uint64_t)blocks_per_wave;
    if (b_end > total_blocks) b_end = total_blocks;

    int idx = 0;
    if (items) {
        int lo = 0, hi = nitems - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (items[mid].block0 <= b_begin) lo = mid; else hi = mid - 1;
        }
        idx = lo;
    }
    CdcItem it = items ? items[idx] : single;
    uint64_t it_end = it.block0 + fnti::cdc_blocks(it.n);
    const CdcTw tw = cdc_twiddles(t);
    int32_t H[4];
    cdc_tap_spectra(items ? &items[idx].taps[0][0] : &single.taps[0][0], it.ntaps, uv, t, tw, H);
    // Eq. (7): z = -2^15 * 64^-1 * IFNT' = -512 IFNT'; Eq. (8): z^ = -2^7 * 64^-1 * IFNT' = -2 IFNT'
    const int32_t scale = uv ? -2 : -512;
    bool have_prev = false;
    uint32_t prev = 0;

    for (uint64_t b = b_begin; b < b_end; ++b) {
        if (b >= it_end) {
            // next item holding block b (skips items with n == 0); a table whose
            // prefix sums do not cover total_blocks ends the wave instead of
            // reading past its last entry
            while (b >= it_end && items && idx + 1 < nitems) {
                ++idx;
                it = items[idx];
                it_end = it.block0 + fnti::cdc_blocks(it.n);
            }
            if (b >= it_end || b < it.block0) return;
            have_prev = false;
            cdc_tap_spectra(&items[idx].taps[0][0], it.ntaps, uv, t, tw, H);
        }
        const int64_t lb = (int64_t)(b - it.block0);
        // window word of instant 32 lb - 32 + lane; lanes 0..31 reuse the
        // previous block's new half when this wave just processed it
        uint32_t carried = (uint32_t)__shfl((int)prev, (lane + 32) & 63);
        uint32_t wd = (have_prev && lane < 32) ? carried : cdc_load(it, 32 * lb - 32 + lane);
        if (!bytes_5bit(wd)) flag(err, RANGE_SAMPLE);
        prev = wd;
        have_prev = true;
        winw[lane] = wd;
        wave_lds_sync();
        int32_t x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t u = winw[t + 16 * j];
            const int32_t xr = sbyte(u, 2 * pol), xi = sbyte(u, 2 * pol + 1);
            x[j] = uv ? xr - 256 * xi : xr + 256 * xi;  // |.| <= 4112
        }
        cdc_fnt64(x, t, tw);
        // P = U H+ (uv = 0 groups), Q = V H- (uv = 1 groups); S = P + Q, D = P - Q
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int32_t pq = mulmod(x[j], H[j]);
            int32_t o = xor_lane<16>(pq);
            x[j] = uv ? o - pq : pq + o;                 // |.| < 2^18
        }
        cdc_ifnt64_upper(x, t, tw);
        const int64_t i0 = 32 * lb;
#pragma unroll
        for (int j = 2; j < 4; ++j) {
            const int32_t z = lift_loose(mulmod(x[j], scale));
            const int il = t + 16 * (j - 2);             // instant within the block
            if (WITH_Z && it.z_out && (uint64_t)(i0 + il) < it.n) it.z_out[(i0 + il) * 4 + g] = z;
            reinterpret_cast<int8_t *>(outw)[il * 4 + g] = (int8_t)clamp32(rs32(z, it.shift), -16, 15);
        }
        wave_lds_sync();
        if (it.a_out && lane < 16) {
            // symbol instants 2 m + phase inside this block
            const int il = 2 * lane + it.phase;
            const int64_t i = i0 + il;
            if ((uint64_t)i < it.n) reinterpret_cast<uint32_t *>(it.a_out)[(i - it.phase) >> 1] = outw[il];
        }
        wave_lds_sync();
    }
}

// ------------------------------------------------------- CDC, lane per block --
//
// One lane computes one whole 32-instant block: the 64-point forward
// transforms of u = x_r + 2^8 x_i and v = x_r - 2^8 x_i (Eqs. (7)-(8) by
// linearity) stay in its registers, with no exchange between lanes.  Only the
// instants the resampler keeps are recovered: for decimation phase 0 the even
// positions 2r of the 64-point inverse are the 32-point inverse (radix
// alpha^2 = 2) of the folded spectrum T[k] = S[k] + S[k + 32]; for phase 1 the
// odd positions are the same inverse of T[k] = alpha^-k (S[k] - S[k + 32]).
// A wave takes CDC_CHUNK consecutive blocks of one channel and first computes
// that channel's tap spectra H+, H- into LDS, one bin per lane.

// Compile-time loop: f(std::integral_constant<int, 0>{}), ..., f(<N - 1>).
template <typename F, int... I>
__device__ __forceinline__ void sfor_(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F &&f) {
    sfor_(f, std::make_integer_sequence<int, N>{});
}

// One fold of a loose residue: 2^16 xh + xl == xl - xh.  Any int32 in, result
// in (-2^15, 2^16 + 2^15).
__device__ __forceinline__ int32_t fold16(int32_t x) {
    return (int32_t)((uint32_t)x & 0xFFFFu) - (x >> 16);
}

// x * 2^e for 1 <= e <= 14, any int32 x: fold, shift (stays below 2^31), fold.
// The shifted value passes through opq so the compiler keeps shift + one SDWA
// subtract instead of rewriting the second fold into mask-and-shift pairs.
__device__ __forceinline__ int32_t mul_pow2(int32_t x, int e) { return fold16(opq(fold16(x) << e)); }

// (a - b) * alpha^E, E a compile-time exponent (alpha = sqrt 2, alpha^(2f) = 2^f,
// 2^16 = -1).  Powers of two below 2^15 take mul_pow2 (any int32 a - b); the
// others take mulmod (|a - b| < 2^23).  Result magnitude < 2^16 + 2^15, or
// |a - b| itself for E = 0, 32.
template <int E>
__device__ __forceinline__ int32_t tw_diff(int32_t a, int32_t b) {
    constexpr int e = E & 63;
    if constexpr (e == 0) {
        return a - b;
    } else if constexpr (e == 32) {
        return b - a;
    } else if constexpr ((e & 1) == 0 && e / 2 < 15) {
        return mul_pow2(a - b, e / 2);
    } else if constexpr ((e & 1) == 0 && e / 2 > 16 && e / 2 < 31) {
        return mul_pow2(b - a, e / 2 - 16);
    } else {
        constexpr AlphaPow tab = make_alpha_pow();
        return mulmod(a - b, opq(tab.v[e]));
    }
}

// Stages h = 16 .. 1 of the 64-point DIF forward transform (radix sqrt 2) on
// one half of the registers.  After the first stage (h = 32) the halves
// x[0..31] (even bins) and x[32..63] (odd bins) are independent 32-point
// transforms with the same twiddles alpha^(j 32 / h); on return x[n] of half
// `hf` holds bin bitrev6(32 hf + n).  In: |x| < 2^16.6; out: |X| < 2^21.6.
template <int H>
__device__ __forceinline__ void fnt64_half_stage(int32_t (&x)[32]) {
    sfor<16 / H>([&](auto gc) {
        constexpr int g = decltype(gc)::value * 2 * H;
        sfor<H>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const int32_t a = x[g + j], b = x[g + j + H];
            x[g + j] = a + b;
            x[g + j + H] = tw_diff<j * (32 / H)>(a, b);
        });
    });
}
__device__ __forceinline__ void fnt64_half(int32_t (&x)[32]) {
    fnt64_half_stage<16>(x);
    fnt64_half_stage<8>(x);
    fnt64_half_stage<4>(x);
    fnt64_half_stage<2>(x);
    fnt64_half_stage<1>(x);
}

// b * 2^-e (mod 65537) subtracted from / added to a, e compile-time in [0, 16):
// 2^-e = -2^(16 - e).  Returns (a + b 2^-e, a - b 2^-e).
template <int E>
__device__ __forceinline__ void inv_bfly(int32_t a, int32_t b, int32_t &lo, int32_t &hi) {
    if constexpr (E == 0) {
        lo = a + b;
        hi = a - b;
    } else if constexpr (E == 1) {
        const int32_t t = mulmod(b, opq(32768));      // b 2^15 = -b 2^-1
        lo = a - t;
        hi = a + t;
    } else {
        const int32_t t = mul_pow2(b, 16 - E);       // b 2^(16-E) = -b 2^-E
        lo = a - t;
        hi = a + t;
    }
}

// 32-point DIT inverse (radix 2, unnormalised), bit-reversed order in; returns
// the natural-order outputs 16..31 in y[16..31].  In: |y| < 2^16.6 (|b| < 2^23
// where mulmod is used); out: |y| < 2^21.6.
template <int H>
__device__ __forceinline__ void ifnt32_stage(int32_t (&y)[32]) {
    sfor<16 / H>([&](auto gc) {
        constexpr int g = decltype(gc)::value * 2 * H;
        sfor<H>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            int32_t lo, hi;
            inv_bfly<j * (16 / H)>(y[g + j], y[g + j + H], lo, hi);
            if constexpr (H < 16) y[g + j] = lo;       // the last stage keeps the upper half
            y[g + j + H] = hi;
        });
    });
}
__device__ __forceinline__ void ifnt32_upper_regs(int32_t (&y)[32]) {
    ifnt32_stage<1>(y);
    ifnt32_stage<2>(y);
    ifnt32_stage<4>(y);
    ifnt32_stage<8>(y);
    ifnt32_stage<16>(y);
}

// Centred value of a loose residue r congruent to a z with |z| <= 32768, for
// |r| < 2^31 - 2^16: fold once into (-2^15, 2^16 + 2^15), where z or z + 65537
// is the only candidate.
__device__ __forceinline__ int32_t lift_z(int32_t r) {
    const int32_t f = fold16(r);
    return f > 32768 ? f - 65537 : f;
}

// rs(z, s) then saturate to 5 bit, for |z| <= 2^16 and 0 <= s <= 16.
__device__ __forceinline__ int32_t requant5(int32_t z, int s) {
    const int32_t r = (z + ((1 << s) >> 1)) >> s;
    return r < -16 ? -16 : (r > 15 ? 15 : r);
}

// Tap spectra of item ip for the lane-per-block CDC, bin k = lane:
// H+- = sum_n (h_r[n] +- 2^8 h_i[n]) alpha^(n k), into hs[0] / hs[1] at the
// register index of bin k (LDS; one wave writes all 64 bins).
__device__ __forceinline__ void cdc_lane_spectra(const CdcItem *ip, int lane, int32_t (*hs)[64]) {
    const int ntaps = ip->ntaps < 32 ? ip->ntaps : 32;
    const int8_t *tp = &ip->taps[0][0];
    const int32_t ak = kAlphaPow.v[lane];
    int32_t a = 1, sr = 0, si = 0;                      // |sums| < 32 * 32 * 2^16.6
    for (int k = 0; k < ntaps; ++k) {
        sr += (int32_t)tp[2 * k] * sext24(a);
        si += (int32_t)tp[2 * k + 1] * sext24(a);
        a = mulmod(a, ak);
    }
    const int32_t r = fold16(sr), i8 = mul_pow2(si, 8);
    const int reg = bitrev(lane, 6);
    hs[0][reg] = r + i8;                               // |.| < 2^17.6
    hs[1][reg] = r - i8;
}

// Overlap-save FNT-CDC of the blocks lb0 + lane of item ip, one whole block per
// lane (hs: the item's tap spectra from cdc_lane_spectra; edge: 2 x 64 words of
// LDS for the windows of edge blocks, private to the wave).  o[q] receives the
// q-th 1-sample/symbol output of the lane's block as 4 packed 5-bit bytes
// {XI, XQ, YI, YQ} (symbol 16 (lb0 + lane) + q).  Returns whether the lane's
// block lies inside the item; lanes past its end compute on zeros.
// With ring16 (an LDS pointer), polarisation p's two output bytes of symbol q
// go straight to ring16[2 (16 lane + q) + p] as each polarisation finishes, and
// o is left untouched (fewer registers live across the two polarisations).
__device__ __forceinline__ bool cdc_lane_blocks(const CdcItem *ip, uint64_t lb0, int lane,
                                                const int32_t (*hs)[64], uint32_t (*edge)[64],
                                                int *err, uint32_t (&o)[16], uint16_t *ring16 = nullptr) {
    const uint64_t n = ip->n;
    const uint64_t nb = fnti::cdc_blocks(n);
    const int shift = ip->shift, phase = ip->phase;
    const int8_t *in = ip->in;
    const int8_t *hist = ip->hist;

    const uint64_t lb = lb0 + (uint64_t)lane;
    const bool active = lb < nb;                        // lanes past the channel's end idle
    const int64_t i0 = 32 * (int64_t)lb - 32;           // first instant of the window
    // interior blocks read their window straight from the input; the first block
    // (history before instant 0) and a partial last block (zeros past n) -- at
    // most two lanes of the wave -- read a copy the wave builds in LDS
    const bool interior = active && lb >= 1 && (uint64_t)(i0 + 64) <= n;
    const uint64_t edges = __ballot(active && !interior);
    const int e0 = edges ? __ffsll((unsigned long long)edges) - 1 : 0;
    const int e1 = edges ? 63 - __clzll((long long)edges) : 0;
    uint32_t bad = 0u;
    for (int k = 0; k < 2; ++k) {                       // uniform: staging of edge windows
        if (k == 1 && e1 == e0) break;
        if (!edges) break;
        const int L = k ? e1 : e0;
        const int64_t i = 32 * (int64_t)(lb0 + L) - 32 + lane;
        uint32_t w = 0u;
        if (i < 0) {
            if (hist) w = reinterpret_cast<const uint32_t *>(hist)[32 + i];
        } else if ((uint64_t)i < n) {
            w = reinterpret_cast<const uint32_t *>(in)[i];
            if (lane >= 32) bad |= w ^ (w << 1);        // new word of block lb0 + L
        }
        edge[k][lane] = w;
    }
    wave_lds_sync();
    // this lane's 64 window words, through a flat pointer into global memory or LDS
    const uint32_t *wp = interior ? reinterpret_cast<const uint32_t *>(in) + i0
                                  : &edge[(active && lane == e1 && e1 != e0) ? 1 : 0][0];
    const bool vec = ((uintptr_t)in & 15u) == 0u;       // uniform: 16-byte loads possible
    if (interior) {                                     // range check of the 32 new words
        if (vec) {
            const uint4 *w4p = reinterpret_cast<const uint4 *>(wp);
#pragma unroll
            for (int q = 8; q < 16; ++q) {
                const uint4 w4 = w4p[q];
                bad |= (w4.x ^ (w4.x << 1)) | (w4.y ^ (w4.y << 1)) | (w4.z ^ (w4.z << 1)) | (w4.w ^ (w4.w << 1));
            }
        } else {
#pragma unroll 8
            for (int q = 32; q < 64; ++q) bad |= wp[q] ^ (wp[q] << 1);
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) o[q] = 0u;
#pragma unroll 1
    for (int pol = 0; pol < 2; ++pol) {
        int32_t ys[32], yd[32];
        sfor<2>([&](auto hc) {
            constexpr int hf = decltype(hc)::value;
            // first DIF stage fused with unpacking: half 0 takes u[j] + u[j + 32],
            // half 1 takes (u[j] - u[j + 32]) alpha^j, u = x_r + 2^8 x_i (v: -)
            int32_t u[32], v[32];
            auto unpack = [&](auto jc, uint32_t w0, uint32_t w1) {
                constexpr int j = decltype(jc)::value;
                // one shift per word brings the polarisation's two bytes down; the
                // byte selects then fold into the adds (SDWA)
                const uint32_t s0 = w0 >> (16 * pol), s1 = w1 >> (16 * pol);
                const int32_t r0 = sbyte(s0, 0), i0b = sbyte(s0, 1);
                const int32_t r1 = sbyte(s1, 0), i1b = sbyte(s1, 1);
                if constexpr (hf == 0) {
                    const int32_t xr = r0 + r1, xi = i0b + i1b;
                    u[j] = xr + 256 * xi;                   // |.| <= 8224
                    v[j] = xr - 256 * xi;
                } else {
                    const int32_t xr = r0 - r1, xi = i0b - i1b;
                    u[j] = tw_diff<j>(xr + 256 * xi, 0);
                    v[j] = tw_diff<j>(xr - 256 * xi, 0);
                }
            };
            if (vec) {
                const uint4 *w4p = reinterpret_cast<const uint4 *>(wp);
                sfor<8>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    const uint4 lo4 = w4p[q], hi4 = w4p[q + 8];
                    unpack(std::integral_constant<int, 4 * q + 0>{}, lo4.x, hi4.x);
                    unpack(std::integral_constant<int, 4 * q + 1>{}, lo4.y, hi4.y);
                    unpack(std::integral_constant<int, 4 * q + 2>{}, lo4.z, hi4.z);
                    unpack(std::integral_constant<int, 4 * q + 3>{}, lo4.w, hi4.w);
                });
            } else {
                sfor<32>([&](auto jc) { unpack(jc, wp[decltype(jc)::value], wp[decltype(jc)::value + 32]); });
            }
            fnt64_half(u);
            fnt64_half(v);
            // P = U H+, Q = V H-; S = P + Q, D = P - Q, folded to the kept phase
#pragma unroll
            for (int r = 0; r < 32; r += 2) {
                const int32_t P0 = mulmod(u[r], hs[0][32 * hf + r]), Q0 = mulmod(v[r], hs[1][32 * hf + r]);
                const int32_t P1 = mulmod(u[r + 1], hs[0][32 * hf + r + 1]);
                const int32_t Q1 = mulmod(v[r + 1], hs[1][32 * hf + r + 1]);
                u[r] = P0 + Q0;                         // |.| < 2^17.4
                v[r] = P0 - Q0;
                u[r + 1] = P1 + Q1;
                v[r + 1] = P1 - Q1;
            }
            if (phase == 0) {
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    ys[16 * hf + m] = fold16(u[2 * m] + u[2 * m + 1]);
                    yd[16 * hf + m] = fold16(v[2 * m] + v[2 * m + 1]);
                }
            } else {
                sfor<16>([&](auto mc) {
                    constexpr int m = 16 * hf + decltype(mc)::value;
                    constexpr int k = ((m & 1) << 4) | ((m & 2) << 2) | (m & 4) | ((m & 8) >> 2) | ((m & 16) >> 4);
                    ys[m] = tw_diff<64 - k>(u[2 * (m - 16 * hf)], u[2 * (m - 16 * hf) + 1]);
                    yd[m] = tw_diff<64 - k>(v[2 * (m - 16 * hf)], v[2 * (m - 16 * hf) + 1]);
                });
            }
            __asm__ volatile("" ::: "memory");          // reload the window for the next pass
        });
        ifnt32_upper_regs(ys);
        ifnt32_upper_regs(yd);
        // Eq. (7): z = -2^15 64^-1 IFNT' = -512 IFNT'; Eq. (8): z^ = -2^7 64^-1 IFNT' = -2 IFNT'
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int32_t zr = lift_z(sext24(ys[16 + q]) * -512);
            const int32_t zi = lift_z(sext24(yd[16 + q]) * -2);
            const uint32_t b2 = ((uint32_t)requant5(zr, shift) & 0xFFu) |
                                (((uint32_t)requant5(zi, shift) & 0xFFu) << 8);
            if (ring16) {
                ((__attribute__((address_space(3))) uint16_t *)ring16)[2 * (16 * lane + q) + pol] = (uint16_t)b2;
            } else {
                o[q] |= b2 << (16 * pol);
            }
        }
    }
    if ((bad & 0xE0E0E0E0u) != 0u) flag(err, RANGE_SAMPLE);
    if (active) count_products(0, 2 * 2 * 64);         // U H+, V H- over 64 bins, both polarisations
    return active;
}

template <int WPG>
__global__ __launch_bounds__(64 * WPG) void cdc_lane_kernel(const CdcItem *items, int nitems,
                                                            CdcItem single, uint64_t total_chunks,
                                                            int *err) {
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    __shared__ int32_t hs_s[WPG][2][64];               // per wave: H+, H- by register index
    __shared__ __align__(16) uint32_t edge_s[WPG][2][64];  // per wave: windows of edge blocks

    const uint64_t chunk = (uint64_t)blockIdx.x * WPG + wv;
    if (chunk >= total_chunks) return;
    int idx = 0;
    if (items) {                                        // last item whose chunk range starts <= chunk
        int lo = 0, hi = nitems - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].chunk0 <= chunk) lo = mid; else hi = mid - 1;
        }
        idx = lo;
    }
    const CdcItem *ip = items ? &items[idx] : &single;
    const uint64_t nb = fnti::cdc_blocks(ip->n);
    const uint64_t lb0 = (chunk - (items ? ip->chunk0 : 0)) * fnti::CDC_CHUNK;
    if (lb0 >= nb) return;                              // a table that does not cover the chunk
    cdc_lane_spectra(ip, lane, hs_s[wv]);
    wave_lds_sync();
    uint32_t o[16];
    const bool active = cdc_lane_blocks(ip, lb0, lane, hs_s[wv], edge_s[wv], err, o);
    int8_t *a_out = ip->a_out;
    if (a_out == nullptr || !active) return;
    const uint64_t M = fnti::n_symbols(ip->n, ip->phase);
    const int64_t m0 = 16 * (int64_t)(lb0 + (uint64_t)lane);   // first symbol of the block
    uint32_t *dst = reinterpret_cast<uint32_t *>(a_out) + m0;
    if ((uint64_t)(m0 + 16) <= M && ((uintptr_t)dst & 15u) == 0u) {
        uint4 *d4 = reinterpret_cast<uint4 *>(dst);
#pragma unroll
        for (int q = 0; q < 4; ++q) d4[q] = make_uint4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
    } else {
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if ((uint64_t)(m0 + q) < M) dst[q] = o[q];
    }
}

// ----------------------------------------------------- CDC, direct comparator --
//
// The same 1-sps 5-bit output by the plain time-domain definition, with no
// Fermat-domain arithmetic: lane m of a wave computes symbol m's four
// components z = sum_k h[k] x[i - k] (i = 2 m + phase) as 4-byte dot products
// of the 32-instant window (stream bytes staged in LDS, stream-major) with the
// taps reversed and packed as int8.  Chunks of 64 blocks per wave, as in
// cdc_lane_kernel; 16 passes of 64 symbols each.
template <int WPG>
__global__ __launch_bounds__(64 * WPG) void cdc_direct_kernel(const CdcItem *items, int nitems,
                                                              CdcItem single, uint64_t total_chunks,
                                                              int *err) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // per wave: 160 staged bytes of each stream (+ 16 pad: the last window's
    // ninth word is read as the ignored high operand of an aligned alignbyte)
    __shared__ __align__(16) uint32_t xb_s[WPG][4][44];
    uint32_t(*xb)[44] = xb_s[wv];
    const uint64_t chunk = (uint64_t)blockIdx.x * WPG + wv;
    if (chunk >= total_chunks) return;
    int idx = 0;
    if (items) {
        int lo = 0, hi = nitems - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].chunk0 <= chunk) lo = mid; else hi = mid - 1;
        }
        idx = lo;
    }
    const CdcItem *ip = items ? &items[idx] : &single;
    const uint64_t n = ip->n;
    const uint64_t lb0 = (chunk - (items ? ip->chunk0 : 0)) * fnti::CDC_CHUNK;
    if (lb0 >= fnti::cdc_blocks(n)) return;
    const int ntaps = ip->ntaps < 32 ? ip->ntaps : 32;
    const int shift = ip->shift, phase = ip->phase;
    const int8_t *in = ip->in;
    const int8_t *hist = ip->hist;
    int8_t *a_out = ip->a_out;
    const uint64_t M = fnti::n_symbols(n, phase);
    // taps reversed (byte t of the window meets h[31 - t]) and packed as int8
    const int8_t *tp = &ip->taps[0][0];
    uint32_t hr[8], hi[8], hn[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        uint32_t r = 0, im = 0, ng = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = 31 - (4 * q + b);
            const int32_t vr = k < ntaps ? tp[2 * k] : 0, vi = k < ntaps ? tp[2 * k + 1] : 0;
            r |= ((uint32_t)vr & 0xFFu) << (8 * b);
            im |= ((uint32_t)vi & 0xFFu) << (8 * b);
            ng |= ((uint32_t)(-vi) & 0xFFu) << (8 * b);
        }
        hr[q] = r;
        hi[q] = im;
        hn[q] = ng;
    }
    uint32_t bad = 0u;
    const int64_t sym0 = 16 * (int64_t)lb0;             // first symbol of the chunk
    for (int sub = 0; sub < fnti::CDC_CHUNK / 4; ++sub) {
        const int64_t s0 = sym0 + 64 * sub;
        if ((uint64_t)s0 >= M) break;
        const int64_t base = 2 * s0 - 32;               // instant at staged byte 0
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int p = lane + 64 * r;
            if (p < 160) {
                const int64_t i = base + p;
                uint32_t w = 0u;
                if (i < 0) {
                    if (hist) w = reinterpret_cast<const uint32_t *>(hist)[32 + i];
                } else if ((uint64_t)i < n) {
                    w = reinterpret_cast<const uint32_t *>(in)[i];
                    if (p >= 32) bad |= w ^ (w << 1);   // instants new to this pass
                }
                uint8_t *xbb = reinterpret_cast<uint8_t *>(&xb[0][0]);
#pragma unroll
                for (int c = 0; c < 4; ++c) xbb[c * 176 + p] = (uint8_t)(w >> (8 * c));
            }
        }
        wave_lds_sync();
        const int64_t m = s0 + lane;
        const int sb = 2 * lane + phase + 1;            // window bytes sb .. sb + 31
        uint32_t o = 0u;
#pragma unroll
        for (int pol = 0; pol < 2; ++pol) {
            uint32_t dr[9], di[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                dr[q] = xb[2 * pol][(sb >> 2) + q];
                di[q] = xb[2 * pol + 1][(sb >> 2) + q];
            }
            int32_t re = 0, im = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int xr = (int)__builtin_amdgcn_alignbyte(dr[q + 1], dr[q], sb & 3);
                const int xi = (int)__builtin_amdgcn_alignbyte(di[q + 1], di[q], sb & 3);
                re = __builtin_amdgcn_sdot4(xr, (int)hr[q], re, false);
                re = __builtin_amdgcn_sdot4(xi, (int)hn[q], re, false);
                im = __builtin_amdgcn_sdot4(xi, (int)hr[q], im, false);
                im = __builtin_amdgcn_sdot4(xr, (int)hi[q], im, false);
            }
            o |= (((uint32_t)requant5(re, shift) & 0xFFu) | (((uint32_t)requant5(im, shift) & 0xFFu) << 8))
                 << (16 * pol);
        }
        if (a_out && (uint64_t)m < M) reinterpret_cast<uint32_t *>(a_out)[m] = o;
    }
    if ((bad & 0xE0E0E0E0u) != 0u) flag(err, RANGE_SAMPLE);
}

// ----------------------------------------------------------------------- AEQ --

__device__ __forceinline__ uint32_t aeq_load(const AeqItem &it, int64_t i, int *err) {
    uint32_t w;
    if (i < 0) {
        w = it.hist_in ? reinterpret_cast<const uint32_t *>(it.hist_in)[16 + i] : 0u;
    } else {
        w = (uint64_t)i < it.m ? gptr(reinterpret_cast<const uint32_t *>(it.a))[i] : 0u;
    }
    if (!bytes_5bit(w)) flag(err, RANGE_SYMBOL);
    return w;
}

// Split the 14-bit tap into two 7-bit digits, w = 2^7 hi + lo with lo in
// [-64, 63] and hi in [-64, 64], pick digit `d` (0 = hi, 1 = lo) and fold in
// N^-1 = 32^-1 = -2048 (mod 65537) so the inverse transform needs no scaling.
__device__ __forceinline__ uint32_t tap_digit(int32_t w, int d) {
    int32_t lo = ((w + 64) & 127) - 64;
    int32_t hi = (w - lo) >> 7;
    return Field<16>::from_int((d ? lo : hi) * -2048);
}

// Final state of one AEQ run: taps, symbol history and CDC history.
__device__ __forceinline__ void aeq_finish(const AeqItem &it, int lane, const int32_t (&w)[4],
                                           int *err) {
    const int s1 = lane >> 4, kk = lane & 15;
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) it.taps[(s1 * 4 + s2) * 16 + kk] = (int16_t)w[s2];
    if (it.hist_out) {
        uint32_t h = (lane < 16) ? aeq_load(it, (int64_t)it.m - 16 + lane, err) : 0u;
        if (lane < 16) reinterpret_cast<uint32_t *>(it.hist_out)[lane] = h;
    }
    if (it.cdc_tail) {
        uint32_t t = 0;
        if (lane < 32) {
            int64_t j = (int64_t)it.cdc_n - 32 + lane;
            t = j >= 0 ? reinterpret_cast<const uint32_t *>(it.cdc_in)[j]
                       : reinterpret_cast<const uint32_t *>(it.cdc_tail)[32 + j];
        }
        if (lane < 32) reinterpret_cast<uint32_t *>(it.cdc_tail)[lane] = t;
    }
}

// Twiddle constants of the N = 32, alpha = 2 transform in the layout where
// lane t (0/1) register j holds position n = t + 2j.  For the radix-2 stage
// with half-size h (h = 16, 8, 4, 2) and the pair starting at register j
// (j' = j mod h/2), the exponent is e = (16/h) t + (32/h) j' < 16.
template <int H, int JP>
__device__ __forceinline__ int32_t tw_fwd(int t) {
    constexpr int e0 = (32 / H) * JP;
    constexpr int e1 = e0 + 16 / H;
    return t ? (1 << e1) : (1 << e0);               // 2^e
}
template <int H, int JP>
__device__ __forceinline__ int32_t tw_inv(int t) {
    constexpr int e0 = (32 / H) * JP;
    constexpr int e1 = e0 + 16 / H;
    // 2^-e = 2^(32 - e) = -2^(16 - e) for 0 < e < 16 (2^16 == -1)
    constexpr int c0 = e0 ? -(1 << (16 - e0)) : 1;
    constexpr int c1 = -(1 << (16 - e1));
    return t ? c1 : c0;
}

// DIF forward transform of 16 tap-digit positions (positions >= 16 are the
// zero padding), two lanes per transform.  In: |x| <= 2^17.  Out: |X| <= 2^21,
// lane t register j holds bin bitrev5(t + 2j).
__device__ __forceinline__ void tap_fnt32(int32_t (&x)[16], int t) {
    // h = 16: the partner positions are zero -> x[j + 8] = x[j] * 2^e
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        int32_t c;
        switch (j) {
            case 0: c = tw_fwd<16, 0>(t); break;
            case 1: c = tw_fwd<16, 1>(t); break;
            case 2: c = tw_fwd<16, 2>(t); break;
            case 3: c = tw_fwd<16, 3>(t); break;
            case 4: c = tw_fwd<16, 4>(t); break;
            case 5: c = tw_fwd<16, 5>(t); break;
            case 6: c = tw_fwd<16, 6>(t); break;
            default: c = tw_fwd<16, 7>(t); break;
        }
        x[j + 8] = mulmod(x[j], c);
    }
    // h = 8, 4, 2: in-register butterflies; sums grow one bit per stage
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j & 4) continue;
        int32_t a = x[j], b = x[j + 4];
        int32_t c;
        switch (j & 3) {
            case 0: c = tw_fwd<8, 0>(t); break;
            case 1: c = tw_fwd<8, 1>(t); break;
            case 2: c = tw_fwd<8, 2>(t); break;
            default: c = tw_fwd<8, 3>(t); break;
        }
        x[j] = a + b;
        x[j + 4] = mulmod(a - b, c);
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j & 2) continue;
        int32_t a = x[j], b = x[j + 2];
        int32_t c = (j & 1) ? tw_fwd<4, 1>(t) : tw_fwd<4, 0>(t);
        x[j] = a + b;
        x[j + 2] = mulmod(a - b, c);
    }
#pragma unroll
    for (int j = 0; j < 16; j += 2) {
        int32_t a = x[j], b = x[j + 1];
        x[j] = a + b;
        x[j + 1] = mulmod(a - b, tw_fwd<2, 0>(t));
    }
    // h = 1: across the lane pair, no twiddle
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        int32_t p = xor_lane<1>(x[j]);
        x[j] = t ? p - x[j] : x[j] + p;
    }
}

// DIT inverse (unnormalised) of 32 bins in the same layout, keeping only the
// outputs at positions 16..31 (registers 8..15).  In: |x| < 2^19.
// Out: |x| < 2^21.
__device__ __forceinline__ void ifnt32_upper(int32_t (&x)[16], int t) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {                  // h = 1: across the lane pair
        int32_t p = xor_lane<1>(x[j]);
        x[j] = t ? p - x[j] : x[j] + p;
    }
#pragma unroll
    for (int j = 0; j < 16; j += 2) {               // h = 2
        int32_t tt = mulmod(x[j + 1], tw_inv<2, 0>(t));
        int32_t a = x[j];
        x[j] = a + tt;
        x[j + 1] = a - tt;
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {                  // h = 4
        if (j & 2) continue;
        int32_t c = (j & 1) ? tw_inv<4, 1>(t) : tw_inv<4, 0>(t);
        int32_t tt = mulmod(x[j + 2], c);
        int32_t a = x[j];
        x[j] = a + tt;
        x[j + 2] = a - tt;
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {                  // h = 8
        if (j & 4) continue;
        int32_t c;
        switch (j & 3) {
            case 0: c = tw_inv<8, 0>(t); break;
            case 1: c = tw_inv<8, 1>(t); break;
            case 2: c = tw_inv<8, 2>(t); break;
            default: c = tw_inv<8, 3>(t); break;
        }
        int32_t tt = mulmod(x[j + 4], c);
        int32_t a = x[j];
        x[j] = a + tt;
        x[j + 4] = a - tt;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {                   // h = 16: upper outputs only
        int32_t c;
        switch (j) {
            case 0: c = tw_inv<16, 0>(t); break;
            case 1: c = tw_inv<16, 1>(t); break;
            case 2: c = tw_inv<16, 2>(t); break;
            case 3: c = tw_inv<16, 3>(t); break;
            case 4: c = tw_inv<16, 4>(t); break;
            case 5: c = tw_inv<16, 5>(t); break;
            case 6: c = tw_inv<16, 6>(t); break;
            default: c = tw_inv<16, 7>(t); break;
        }
        x[j + 8] = x[j] - mulmod(x[j + 8], c);
    }
}

// FNT-AEQ, one wave64 per channel.  Lane roles:
//  * transform lanes: t = bit 0, s = bit 1, d = bit 2, S2 = bits 3-4, g = bit 5;
//    the lane pair (t = 0, 1) holds the 32 bins of filter (S1 = 2g + s, S2),
//    tap digit d (0 = high, 1 = low), 16 bins per lane.
//  * input-spectrum lanes: S1 = lane / 16, 2 of the 32 window positions each.
//  * output / error lanes: symbol m = lane / 4, stream S2 = lane % 4.
//  * gradient / tap-state lanes: S1 = lane / 16, tap k = lane % 16, all 4 S2.
//
// FDG selects how the RDE gradient of the block update (Eq. (6)) is formed:
// false, 4-byte dot products over the window (as every other AEQ kernel);
// true, in the Fermat domain as well.  G[k] = sum_m eps[m] x[16 b + m - k]
// (k < 16) is a correlation of the block's 16 error terms with the 32-symbol
// window: with e'[n] = eps[15 - n] (n < 16, zero above) the cyclic convolution
// c = IFNT(FNT(window) FNT(e')) has c[31 - k] = G[k] with no wrap-around, and
// every true value is within 16 * 128 * 16 = 32768 = (F - 1) / 2 (Eq. (5)), so
// the centred lift is exact.  The window spectra are the ones the filtering
// already computed; per block this adds four error transforms, 512 spectral
// products and 16 inverse transforms (upper halves).
template <bool FDG>
__global__ __launch_bounds__(64) void aeq_fnt_kernel(const AeqItem *items, AeqItem single,
                                                     int *err) {
    const AeqItem it = items ? items[blockIdx.x] : single;
    const int lane = threadIdx.x;
    const int pos = lane & 31;
    const int t = lane & 1, s = (lane >> 1) & 1, d = (lane >> 2) & 1;
    const int tS2 = (lane >> 3) & 3, g = lane >> 5;
    const int tS1 = 2 * g + s;
    const int s1 = lane >> 4, kk = lane & 15;        // gradient / A-spectrum / tap-state role
    const int om = lane >> 2, oS2 = lane & 3;         // output / error role

    __shared__ int16_t tapl[256];                     // [S1][S2][k]
    __shared__ int32_t aspec[4][32];                  // input spectra by position
    __shared__ int32_t part[4][64];                   // [g*2+d][m*4+S2] lifted partial outputs
    __shared__ uint32_t epsw[16];                     // bytes [S2][m]
    __shared__ uint32_t winw[36];                     // bytes [S1][32] window + zero pad
    __shared__ int32_t espec[FDG ? 4 : 1][32];        // error spectra by position (FDG)
    __shared__ int32_t gl[FDG ? 256 : 1];             // gradient [S1][S2][k] (FDG)

    int32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int32_t v = it.taps[(s1 * 4 + q) * 16 + kk];
        if (v < -8192 || v > 8191) flag(err, RANGE_TAP);
        w[q] = clamp32(v, -8192, 8191);
    }
    const uint64_t M = it.m;
    if (M == 0) {
        aeq_finish(it, lane, w, err);
        return;
    }
    if (lane < 4) winw[32 + lane] = 0u;

    // tap-digit spectra of filter (tS1, tS2), digit d, with N^-1 = -2048 folded in
    int32_t W[16];
    auto transform_taps = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) tapl[(s1 * 4 + q) * 16 + kk] = (int16_t)w[q];
        __syncthreads();
        const int base = (tS1 * 4 + tS2) * 16 + t;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            int32_t v = tapl[base + 2 * j];
            int32_t lo = ((v + 64) & 127) - 64;
            int32_t hi = (v - lo) >> 7;
            W[j] = (d ? lo : hi) * -2048;             // |.| <= 64 * 2048 = 2^17
        }
        tap_fnt32(W, t);
        __syncthreads();
    };
    transform_taps();

    const int64_t nblocks = (int64_t)((M + 15) / 16);
    const int c2 = it.const_unit * it.const_unit;
    uint32_t win = aeq_load(it, -16 + pos, err);      // lane pos: symbol 16 b - 16 + pos

    // FNT32 (alpha = 2) of 16 sequences spread over 16 lanes each: lane (s1, kk)
    // enters positions kk and kk + 16 and leaves with the bins stored at kk and
    // kk + 16 of its row (the order the tap-digit spectra use).  |x| <= 128:
    // out |.| <= 2^21.
    auto spectrum = [&](int32_t x0, int32_t x1, int32_t &u0, int32_t &u1) {
        u0 = x0 + x1;
        u1 = mulmod(x0 - x1, 1 << kk);                // h = 16, e = kk
#pragma unroll
        for (int h = 8; h >= 1; h >>= 1) {
            const bool up = (kk & h) != 0;
            const int32_t c = 1 << ((16 / h) * (kk & (h - 1)));
            int32_t p0 = h == 8 ? xor_lane<8>(u0) : h == 4 ? xor_lane<4>(u0)
                       : h == 2 ? xor_lane<2>(u0) : xor_lane<1>(u0);
            int32_t p1 = h == 8 ? xor_lane<8>(u1) : h == 4 ? xor_lane<4>(u1)
                       : h == 2 ? xor_lane<2>(u1) : xor_lane<1>(u1);
            u0 = blend(up, mulmod(p0 - u0, c), u0 + p0);
            u1 = blend(up, mulmod(p1 - u1, c), u1 + p1);
        }
    };

    for (int64_t b = 0; b < nblocks; ++b) {
        uint32_t nxt = pos >= 16 ? aeq_load(it, 16 * b + pos, err) : 0u;
        if (lane < 32) {
            uint8_t *wb = reinterpret_cast<uint8_t *>(winw);
#pragma unroll
            for (int c = 0; c < 4; ++c) wb[c * 32 + pos] = (uint8_t)(win >> (8 * c));
        }
        __syncthreads();
        // input spectra: lane (s1, kk) holds positions kk and kk + 16 of stream s1
        {
            const int8_t *wb = reinterpret_cast<const int8_t *>(winw) + s1 * 32;
            int32_t u0, u1;
            spectrum(wb[kk], wb[kk + 16], u0, u1);
            aspec[s1][kk] = u0;                        // |.| <= 2^21
            aspec[s1][kk + 16] = u1;
        }
        __syncthreads();
        // Fermat-domain 4x4 MIMO: product with the tap-digit spectra; the two
        // streams of a polarisation are summed before one inverse transform
        // (Eq. (5): 2 streams * 16 taps * 64 * 16 = 32768 = (F - 1) / 2)
        int32_t Y[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            int32_t P = mulmod(aspec[tS1][t + 2 * j], W[j]);
            Y[j] = P + xor_lane<2>(P);                 // |.| < 2^18
        }
        ifnt32_upper(Y, t);
        if (s == 0) {
#pragma unroll
            for (int j = 8; j < 16; ++j)
                part[g * 2 + d][(t + 2 * (j - 8)) * 4 + tS2] = lift_loose(Y[j]);
        }
        __syncthreads();
        // recombine the digit groups and the polarisation pairs: one (m, S2) per lane
        const int32_t y = 128 * (part[0][lane] + part[2][lane]) + part[1][lane] + part[3][lane];
        const int32_t yh = (int32_t)clamp64(rs64((int64_t)y, it.out_shift), -32768, 32767);
        const int64_t m = 16 * b + om;
        const bool valid = (uint64_t)m < M;
        if (valid) gptr(it.out)[m * 4 + oS2] = (int16_t)yh;
        if (it.update_enable) {
            // RDE error of this symbol's polarisation and the 8-bit error term
            const int32_t yp = xor_lane<1>(yh);
            const int64_t r2 = (int64_t)yh * yh + (int64_t)yp * yp;
            const int64_t R2 = r2 < 6LL * c2 ? 2LL * c2 : (r2 < 14LL * c2 ? 10LL * c2 : 18LL * c2);
            int32_t eps = (int32_t)clamp64(rs64((R2 - r2) * yh, it.err_shift), -128, 127);
            if (!valid) eps = 0;
            reinterpret_cast<int8_t *>(epsw)[oS2 * 16 + om] = (int8_t)eps;
            __syncthreads();
            if constexpr (FDG) {
                // error spectra: lane (S2 = s1, kk) enters e'[kk] = eps_S2[15 - kk], e'[kk + 16] = 0
                {
                    const int8_t *eb = reinterpret_cast<const int8_t *>(epsw) + s1 * 16;
                    int32_t u0, u1;
                    spectrum(eb[15 - kk], 0, u0, u1);
                    espec[s1][kk] = u0;
                    espec[s1][kk + 16] = u1;
                }
                __syncthreads();
                // filter (S1 = tS1, S2 = tS2) on the lane pair t (both digit lanes
                // compute it; d = 0 keeps it): products |.| < 2^17, inverse upper half
                int32_t C[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) C[j] = mulmod(aspec[tS1][t + 2 * j], espec[tS2][t + 2 * j]);
                ifnt32_upper(C, t);                    // |.| < 2^21
                if (d == 0) {
                    // register j >= 8 holds c[16 + t + 2 (j - 8)] = G[15 - t - 2 (j - 8)]; N^-1 = -2048
#pragma unroll
                    for (int j = 8; j < 16; ++j)
                        gl[(tS1 * 4 + tS2) * 16 + 15 - t - 2 * (j - 8)] = lift_loose(mulmod(C[j], -2048));
                }
                __syncthreads();
#pragma unroll
                for (int q2 = 0; q2 < 4; ++q2) {
                    const int32_t g = gl[(s1 * 4 + q2) * 16 + kk];
                    w[q2] = clamp32(w[q2] + (int32_t)rs64((int64_t)g, step_shift(it, it.block0 + (uint64_t)b)), -8192, 8191);
                }
                transform_taps();
            } else {
            // G[S1][S2][k] = sum_j eps_S2[j] * a_S1[16 b + j - k] as 4-byte dot products
            const int off = s1 * 32 + 16 - kk;
            uint32_t dd[5];
#pragma unroll
            for (int r = 0; r < 5; ++r) dd[r] = winw[(off >> 2) + r];
            uint32_t xs[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) xs[q] = __builtin_amdgcn_alignbyte(dd[q + 1], dd[q], off & 3);
#pragma unroll
            for (int q2 = 0; q2 < 4; ++q2) {
                int32_t gsum = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    gsum = __builtin_amdgcn_sdot4((int)epsw[q2 * 4 + q], (int)xs[q], gsum, false);
                w[q2] = clamp32(w[q2] + (int32_t)rs64((int64_t)gsum, step_shift(it, it.block0 + (uint64_t)b)), -8192, 8191);
            }
            transform_taps();
            }
        } else {
            __syncthreads();
        }
        uint32_t slid = (uint32_t)__shfl((int)win, (lane & 32) | ((pos + 16) & 31));
        win = pos < 16 ? slid : nxt;
    }
    aeq_finish(it, lane, w, err);
}

// ------------------------------------------------------------------------
// FNT-AEQ split by output polarisation.
//
// The outputs of polarisation P (streams S2 = 2P, 2P+1) depend only on the 8
// filters (S1 = 0..3) -> S2, and the RDE error of Eq. (6) for those filters
// only on the same two outputs, so the 4x4 equaliser separates exactly into
// two independent 4x2 halves.  One workgroup runs one half of one channel,
// with WPP = LPT / 4 waves:
//   * 16 tap-digit transforms per half (4 S1 x 2 S2 x 2 digits) over 64*WPP
//     lanes: LPT lanes per transform, PPL = 32 / LPT bins per lane, lane t of a
//     group holding positions n = t + LPT*j (stages with h >= LPT stay in
//     registers, the rest exchange lanes t ^ h);
//   * WPP = 2 splits the two tap digits over the waves, WPP = 4 also the two
//     stream pairs (XI,XQ) / (YI,YQ); the waves then meet once per block to sum
//     their partial outputs.
// ------------------------------------------------------------------------
// The same bin of the partner transform (S1 = 2g + 1 for S1 = 2g), LPT lanes
// further on.  For LPT = 4 the lanes that keep the pair sum (even transforms:
// lanes 0-3 and 8-11 of every row of 16) read lane + 4 by a DPP row rotation;
// the odd transforms' sums are discarded.
template <int LPT>
__device__ __forceinline__ int32_t s1_partner(int32_t v) {
    if constexpr (LPT == 4) return __builtin_amdgcn_update_dpp(0, v, 0x12C, 0xF, 0xF, true);   // row_ror:12
    else return xor_lane<LPT>(v);
}

template <int H>
__device__ __forceinline__ int32_t xor_h(int32_t v) { return xor_lane<H>(v); }

// One butterfly of a cross-lane stage at distance H with its twiddle folded in:
// fold16(x a + p b), p the partner lane's value, for per-lane constants a, b
// that give the lower and the upper lane of a pair their own outputs.  Two
// 24-bit multiplies (the partner's value enters the first through DPP) and one
// fold.  Needs |x|, |p| < 2^23 and |x a| + |p b| < 2^31; the result has
// magnitude < 2^16 + 2^15.  The partner product passes through opq so that it
// stays a multiply of its own (which takes the DPP operand) instead of being
// merged into the multiply-add.
template <int H>
__device__ __forceinline__ int32_t xbfly(int32_t x, int32_t a, int32_t b) {
    const int32_t q = opq(sext24(xor_pos<H>(x)) * sext24(b));
    return fold16(sext24(x) * sext24(a) + q);
}

// Per-lane constants (a, b) of xbfly for the cross-lane stages of one
// transform lane.  DIF stage at distance h: lower lane x + p, upper lane
// (p - x) 2^e.  DIT stage: lower lane x + w p, upper lane p - w x with
// w = 2^-e (= -2^(16-e), or 1 for e = 0).
struct XbCoef { int32_t a, b; };
__device__ __forceinline__ XbCoef xb_dif(int t, int h) {
    const bool up = (t & h) != 0;
    const int32_t c = 1 << ((16 / h) * (t & (h - 1)));
    return {opq(up ? -c : 1), opq(up ? c : 1)};
}
__device__ __forceinline__ XbCoef xb_dit(int t, int h) {
    const bool up = (t & h) != 0;
    const int e = (16 / h) * (t & (h - 1));
    const int32_t w = e ? -(1 << (16 - e)) : 1;
    return {opq(up ? -w : 1), opq(up ? 1 : w)};
}

// 2^-e (mod 65537) as a small signed constant, 0 <= e < 16.
__device__ __forceinline__ int32_t inv_pow2(int e) { return e ? -(1 << (16 - e)) : 1; }

// -2048 2^e (mod 65537) as a small signed constant, 0 <= e < 16: -2^(11+e)
// for e <= 4, 2^(e-5) above (2^16 = -1).
__device__ __forceinline__ int32_t ninv32_pow2(int e) { return e <= 4 ? -(1 << (11 + e)) : 1 << (e - 5); }

// Every twiddle and sign a lane of the polarisation-split AEQ applies, computed
// once before the block loop (lane position t of its transform, kp of its
// input-spectrum group).  The values pass through opq: the compiler must not
// see powers of two and rewrite the multiplies into longer shift sequences.
template <int LPT>
struct PolLaneK {
    static constexpr int NT = 16 / LPT;
    XbCoef tap2;               // tap transform, distance 2
    XbCoef inv[3];             // inverse, distances 2, 4, 8
    XbCoef spec[3];            // input spectra, distances 8, 4, 2
    int32_t sg, sgk;           // +-1 by t & 1 and by kp & 1 (distance-1 stages)
    int32_t h16[NT];           // tap transform, first stage: -2048 2^(t + LPT j)
    int32_t n2048;             // -2048 = 32^-1
    int32_t iw_first;          // inverse, first in-register stage (h = LPT < 16): 2^-(16/LPT) t
    int32_t iw_second;         // inverse, h = 2 LPT < 16, j even: 2^-(8/LPT) t
    int32_t iw_last;           // inverse, h = 16, j = 0: 2^-t
    __device__ __forceinline__ PolLaneK(int t, int kp) {
        tap2 = xb_dif(t, 2);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            inv[i] = xb_dit(t, 2 << i);
            spec[i] = xb_dif(kp, 8 >> i);
        }
        sg = opq((t & 1) ? -1 : 1);
        sgk = opq((kp & 1) ? -1 : 1);
#pragma unroll
        for (int j = 0; j < NT; ++j) h16[j] = opq(ninv32_pow2(t + LPT * j));
        n2048 = opq(-2048);
        iw_first = opq(inv_pow2((16 / LPT) * t));
        iw_second = opq(inv_pow2(((16 / (2 * LPT)) * t) & 15));
        iw_last = opq(inv_pow2(t));
    }
};

// x * s for |x| < 2^23 and a lane constant s (24-bit product).
__device__ __forceinline__ int32_t mul24k(int32_t x, int32_t s) { return sext24(x) * sext24(s); }

// In-register and cross-lane DIF of 16 tap digits zero-padded to 32, times
// 32^-1 = -2048 (so the inverse needs no scaling).  In: digits |d| <= 64 in
// x[0 .. NT-1]; out: |X| < 2^18; register j of lane t holds bin bitrev5(t + LPT j).
// The first stage (partner zero padding) is one 24-bit multiply per output:
// d (-2048), and d (-2048) 2^e as a small constant; later in-register twiddles
// are shifts (mul_pow2, every lane's exponent <= 14); distance 2 across lanes is
// xbfly, distance 4 and 8 keep the shift form (digit sums of up to 2^18 times
// 2^12 leave no headroom there), distance 1 is a signed sum.
template <int LPT>
__device__ __forceinline__ void tap_fnt_lpt(int32_t (&x)[32 / LPT], int t, const PolLaneK<LPT> &k) {
    constexpr int PPL = 32 / LPT;
    constexpr int NT = PPL / 2;
#pragma unroll
    for (int j = 0; j < NT; ++j) {              // h = 16: |d 2^(11+e)| <= 2^21
        x[j + NT] = mul24k(x[j], k.h16[j]);
        x[j] = mul24k(x[j], k.n2048);             // |.| <= 2^17
    }
#pragma unroll
    for (int h = 8; h >= LPT; h >>= 1) {
        const int jd = h / LPT;
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            if (j & jd) continue;
            const int jp = j & (jd - 1);
            const int e = (16 / h) * t + (16 * LPT / h) * jp;               // <= 14
            int32_t a = x[j], b = x[j + jd];
            x[j] = a + b;
            x[j + jd] = mul_pow2(a - b, e);
        }
    }
    // across lanes: lower lane x + p, upper lane (p - x) * 2^e, e <= 14
#pragma unroll
    for (int h = LPT / 2; h >= 2; h >>= 1) {
        if (h == 2) {
#pragma unroll
            for (int j = 0; j < PPL; ++j) x[j] = xbfly<2>(x[j], k.tap2.a, k.tap2.b);
        } else {
            const bool up = (t & h) != 0;
            const int e = (16 / h) * (t & (h - 1));
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                int32_t p = h == 8 ? xor_pos<8>(x[j]) : xor_pos<4>(x[j]);
                x[j] = blend(up, mul_pow2(p - x[j], e), x[j] + p);
            }
        }
    }
    // distance 1, twiddle 1: lower lane p + x, upper lane p - x  (|x| < 2^17)
#pragma unroll
    for (int j = 0; j < PPL; ++j) x[j] = xor_pos<1>(x[j]) + mul24k(x[j], k.sg);
}

// DIT inverse (unnormalised) keeping positions 16..31 (registers PPL/2..PPL-1).
// In: |x| < 2^18; out: any int32 (a loose residue for lift_loose).
// Distance 1 is a signed sum; the other cross-lane stages are xbfly (outputs
// < 2^16.6).  The first in-register stage multiplies by w = 2^-e directly
// (|w| <= 2^14, outputs < 2^30.6); at h = 2 LPT < 16 the registers whose
// exponent can be 0 fold the operand and multiply likewise (outputs < 2^31),
// the others take the shift form; at h = 16 the exponent can be 1 (w = -2^15)
// in the first register: mulmod on the folded operand, shift form elsewhere.
template <int LPT>
__device__ __forceinline__ void ifnt_upper_lpt(int32_t (&x)[32 / LPT], int t, const PolLaneK<LPT> &k) {
    constexpr int PPL = 32 / LPT;
#pragma unroll
    for (int j = 0; j < PPL; ++j) x[j] = xor_pos<1>(x[j]) + mul24k(x[j], k.sg);     // |.| < 2^18.4
#pragma unroll
    for (int h = 2, hi = 0; h < LPT; h <<= 1, ++hi) {
#pragma unroll
        for (int j = 0; j < PPL; ++j)
            x[j] = h == 8 ? xbfly<8>(x[j], k.inv[hi].a, k.inv[hi].b)
                 : h == 4 ? xbfly<4>(x[j], k.inv[hi].a, k.inv[hi].b)
                          : xbfly<2>(x[j], k.inv[hi].a, k.inv[hi].b);
    }
#pragma unroll
    for (int h = LPT; h <= 16; h <<= 1) {
        const int jd = h / LPT;
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            if (j & jd) continue;
            const int jp = j & (jd - 1);
            const int e = (16 / h) * t + (16 * LPT / h) * jp;
            const int32_t a = x[j];
            if (h < 16 && (h == LPT || jp == 0)) {
                // tt = b w: |b| < 2^16.6 (first stage) or folded, |w| <= 2^14
                const int32_t b = h == LPT ? x[j + jd] : fold16(x[j + jd]);
                const int32_t tt = mul24k(b, h == LPT ? k.iw_first : k.iw_second);
                x[j] = a + tt;
                x[j + jd] = a - tt;
            } else if ((16 * LPT / h) * jp >= 2) {
                // every lane has 2 <= e: tt = -m with m = x 2^(16-e), 16 - e <= 14
                const int32_t m = mul_pow2(x[j + jd], 16 - e);
                if (h == 16) {
                    x[j + jd] = a + m;                // only the upper half is kept
                } else {
                    x[j] = a - m;
                    x[j + jd] = a + m;
                }
            } else {                                  // h = 16, j = 0: w = 2^-t
                const int32_t b = h == LPT ? x[j + jd] : fold16(x[j + jd]);
                x[j + jd] = a - mulmod(b, k.iw_last);
            }
        }
    }
}

// Symbol i of the AEQ input (history before 0, zeros past m), as one dword.
__device__ __forceinline__ uint32_t aeq_sym(const AeqItem &it, int64_t i) {
    uint32_t v = 0u;
    if (i < 0) {
        if (it.hist_in != nullptr && i >= -16) v = reinterpret_cast<const uint32_t *>(it.hist_in)[16 + i];
    } else if ((uint64_t)i < it.m) {
        v = reinterpret_cast<const uint32_t *>(it.a)[i];
    }
    return v;
}

// Workgroups of the polarisation-split AEQ: each run of 16 workgroup indices
// holds 8 channels, the two halves of a channel 8 indices apart.  Workgroups
// are dealt round-robin over the 8 XCDs, so both halves of a channel run on one
// XCD and share its L2: the input window both read, and the output records
// whose 16-bit pieces both write, then cross HBM once.
__host__ __device__ constexpr unsigned pol_blocks(int n) { return 16u * (unsigned)((n + 7) / 8); }

// Where the polarisation-split AEQ reads its 1-sample/symbol input.  Every
// source gives symbol i of the channel's stream (history before 0, zeros past
// M) for the two window loads before the first block (first), the window of
// block b + 2 loaded during block b (ahead: symbols 16 b + 16 .. 16 b + 47,
// index clamped to M - 1).  A segmented source is told before the blocks
// [b0, b1) of a segment run (segment) and after (segment_done).
struct AeqSrcGlobal {          // the stream in device memory
    const AeqItem *it;
    __attribute__((address_space(1))) const uint32_t *base;
    uint64_t M;
    __device__ __forceinline__ void prime() {}
    __device__ __forceinline__ uint32_t first(int64_t i) const { return aeq_sym(*it, i); }
    __device__ __forceinline__ uint32_t ahead(uint32_t b, int wpos) {
        return base[min<uint64_t>(16 * (uint64_t)b + 16 + wpos, M - 1)];
    }
    static constexpr bool kSegmented = false;
    __device__ __forceinline__ void segment(uint32_t, uint32_t) {}
    __device__ __forceinline__ void segment_done(uint32_t) {}
};

// Counters of the fused kernel's hand-offs live in LDS and are read and
// written with workgroup-scope atomics (on gfx950: plain LDS loads and stores
// with lgkmcnt waits).  A wait polls with s_sleep between reads and gives up
// after `limit` polls, or when another wave of the workgroup has given up (the
// workgroup's `stall` word, looked at every 64 polls): it then latches RANGE_STALL, sets `stall`
// and reports false, and no wave of the workgroup waits again for the rest of
// the launch, so every wave still ends.  Polls sleep about 64 * SLEEP cycles
// each; with the limits the launchers pass a give-up takes seconds, far beyond
// any legitimate wait (a chunk of CDC or a few blocks of AEQ, microseconds).
// The loaded word is the same for every lane; readfirstlane tells the compiler
// so, and the waits become scalar branches instead of exec-masked loops.
__device__ __forceinline__ uint32_t lds_load_acq(const uint32_t *p) {
    return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
}
__device__ __forceinline__ void lds_store_rel(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <int SLEEP>
__device__ __forceinline__ bool wait_at_least(const uint32_t *p, uint32_t target, uint32_t limit, int *err,
                                              uint32_t *stall, uint32_t *seen = nullptr) {
    uint32_t polls = 0, v;
    while ((v = lds_load_acq(p)) < target) {
        if ((++polls & 63) == 0 &&
            (polls > limit || __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                                  stall, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) != 0u)) {
            flag(err, RANGE_STALL);
            __hip_atomic_store(stall, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return false;
        }
        if constexpr (SLEEP > 0) __builtin_amdgcn_s_sleep(SLEEP);
    }
    if (seen) *seen = v;
    return true;
}

// Ring of CDC output in LDS: RING chunks of 64 CDC blocks (1024 symbols, 4 KB)
// each; symbol i of the channel sits at word i mod (RING * 1024).  Word s of
// `slots` holds 1 + the index of the chunk slot s contains (0: none yet).
constexpr int FUSED_CHUNK_SYMS = 16 * fnti::CDC_CHUNK;

template <int RING>
struct AeqSrcRing {            // the CDC output ring of the fused kernel
    static constexpr uint32_t WORDS = RING * FUSED_CHUNK_SYMS;
    const AeqItem *it;
    const uint32_t *ring;      // LDS, WORDS words
    const uint32_t *slots;     // LDS, RING words
    uint32_t *mine;            // LDS: blocks this wave has finished
    uint32_t *stall;           // LDS: set once a wait of the workgroup gave up
    uint64_t M;
    uint32_t limit;
    int *err;
    uint32_t have;             // chunks [0, have) known to be written (wave-uniform)
    bool live;                 // false once a wait gave up
    // the other polarisation half's progress words in the same workgroup (none
    // when a workgroup runs one half)
    const uint32_t *peer = nullptr;
    int npeer = 0;
    // chunks complete out of order when several producer waves share them out,
    // so each is checked in its own slot, in order
    __device__ __forceinline__ void need(uint32_t chunk) {
        while (have <= chunk && live) {
            live = wait_at_least<2>(&slots[have % RING], have + 1, limit, err, stall);
            ++have;
        }
    }
    static constexpr bool kSegmented = true;
    __device__ __forceinline__ void prime() { need(0); }
    __device__ __forceinline__ uint32_t first(int64_t i) const {
        if (i < 0) return aeq_sym(*it, i);
        return (uint64_t)i < M ? ring[i & (WORDS - 1)] : 0u;
    }
    // Before the blocks [b0, b1): every chunk they read ahead, checked once; and
    // the other half done with the blocks before b0, so that the halves stay
    // within one segment of each other.  The two halves write the 16-bit pieces
    // of the same output records: apart by up to the ring's length, partial
    // lines left the L2 cache before the other half filled them, and the kernel
    // wrote 1.6 times its output bytes.  The slower half never waits for the
    // faster one, and the channel ends with the slower half anyway.
    __device__ __forceinline__ void segment(uint32_t b0, uint32_t b1) {
        for (int k = 0; k < npeer; ++k)
            if (live) live = wait_at_least<2>(&peer[k], b0, limit, err, stall);
        need((uint32_t)(min<uint64_t>(16 * (uint64_t)(b1 - 1) + 47, M - 1) / FUSED_CHUNK_SYMS));
    }
    __device__ __forceinline__ uint32_t ahead(uint32_t b, int wpos) const {
        return ring[min<uint64_t>(16 * (uint64_t)b + 16 + wpos, M - 1) & (WORDS - 1)];
    }
    // the blocks before b1 are done: published for the producers
    __device__ __forceinline__ void segment_done(uint32_t b1) {
        if ((threadIdx.x & 63) == 0) lds_store_rel(mine, b1);
    }
};

// Barrier of the WPP waves of one polarisation half, once per block.  Plain
// launches use the workgroup barrier (a workgroup is one half); the fused
// kernel holds both halves and the producer waves, so a half's waves meet in
// LDS instead: wave vh writes 1 + the block it finished into its own word of
// the half (after its partial outputs) and waits until every word of the half
// has reached that block (one LDS load of all WPP words per poll).
struct HalfSyncWg {
    __device__ __forceinline__ void block(uint32_t) { __syncthreads(); }
};
template <int WPP>
struct HalfSyncLds {
    uint32_t *arrive;          // LDS, WPP words of this half, zeroed before the channel
    uint32_t *stall;           // LDS: set once a wait of the workgroup gave up
    uint32_t limit;
    int *err;
    int vh;
    bool live;
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    // one LDS load of the half's words (the pointer is cast to the LDS address
    // space: through a generic pointer a volatile load would be a flat load)
    __device__ __forceinline__ uint32_t slowest() const {
        if constexpr (WPP == 2) {
            const u32x2 a = *(const volatile __attribute__((address_space(3))) u32x2 *)arrive;
            return __builtin_amdgcn_readfirstlane(min(a.x, a.y));
        } else {
            const u32x4 a = *(const volatile __attribute__((address_space(3))) u32x4 *)arrive;
            return __builtin_amdgcn_readfirstlane(min(min(a.x, a.y), min(a.z, a.w)));
        }
    }
    __device__ __forceinline__ void block(uint32_t b) {
        if ((threadIdx.x & 63) == 0) lds_store_rel(&arrive[vh], b + 1);   // after the partial outputs
        if (!live) return;
        uint32_t polls = 0;
        while (slowest() < b + 1) {
            if ((++polls & 63) == 0 &&
                (polls > limit || __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                                      stall, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) != 0u)) {
                flag(err, RANGE_STALL);
                __hip_atomic_store(stall, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                live = false;
                return;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");   // the partial outputs after the words
    }
};

// The AEQ of one channel in the polarisation-split form: this wave is wave vh
// of the WPP = LPT / 4 waves of half `pol`.  LDS of the wave: aspec (input
// spectra, two buffers by block parity), epsw (error bytes), winw (window
// bytes); of the half: part_h
// (partial outputs, by block parity).  Reads its input through src and meets
// the other waves of its half through hsync once per block.
template <int LPT, class Src, class Sync>
__device__ __forceinline__ void aeq_pol_run(const AeqItem &it, int pol, int vh, int lane, int *err,
                                            int32_t (*aspec)[4][kSpecRow], int32_t (*part_h)[4][33], uint32_t *epsw,
                                            uint32_t *winw, Src &src, Sync &hsync) {
    constexpr int WPP = LPT / 4;                       // waves per polarisation half
    constexpr int PPL = 32 / LPT;                      // bins per lane
    constexpr int NT = 16 / LPT;                       // taps owned per lane (= PPL / 2)
    // transform role: filter (tS1 -> 2 pol + tS2l), digit td, lane t of LPT; the
    // lane also owns the taps k = t + LPT i (i < NT) of that filter
    const int tr = lane / LPT, t = lane_pos(lane % LPT);
    const int ts = tr & 1, tS2l = (tr >> 1) & 1;
    const int td = WPP == 1 ? (tr >> 2) & 1 : (vh & 1);
    const int tg = WPP == 1 ? (tr >> 3) : WPP == 2 ? (tr >> 2) & 1 : (vh >> 1);
    const int tS1 = 2 * tg + ts;
    const int tS2 = 2 * pol + tS2l;
    // output / error role (lanes 0..31 of every wave): symbol om, stream 2 pol + oS2l
    const int om = (lane >> 1) & 15, oS2l = lane & 1;
    const int kk = lane & 15;

    int16_t *const wrow = it.taps + (tS1 * 4 + tS2) * 16;
    int32_t w[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        int32_t val = wrow[t + LPT * i];
        if (val < -8192 || val > 8191) flag(err, RANGE_TAP);
        w[i] = clamp32(val, -8192, 8191);
    }
    // M and the block count are the same for every lane; readfirstlane keeps them
    // (and the block loop's counter) in scalar registers whatever way the item
    // reached this wave
    const uint64_t M = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(it.m >> 32)) << 32) |
                       __builtin_amdgcn_readfirstlane((uint32_t)it.m);
    const bool writer = vh == 0;                       // stores the outputs
    const bool tap_owner = td == 0;                    // one of the two digit copies stores taps
    const bool hist_owner = pol == 0 && vh == 0;
    auto finish = [&]() {
        if (tap_owner) {
#pragma unroll
            for (int i = 0; i < NT; ++i) wrow[t + LPT * i] = (int16_t)w[i];
        }
        if (hist_owner) {
            if (it.hist_out) {
                uint32_t h = (lane < 16) ? src.first((int64_t)M - 16 + lane) : 0u;
                if (lane < 16) reinterpret_cast<uint32_t *>(it.hist_out)[lane] = h;
            }
            if (it.cdc_tail) {
                uint32_t tl = 0;
                if (lane < 32) {
                    int64_t j = (int64_t)it.cdc_n - 32 + lane;
                    tl = j >= 0 ? reinterpret_cast<const uint32_t *>(it.cdc_in)[j]
                                : reinterpret_cast<const uint32_t *>(it.cdc_tail)[32 + j];
                }
                if (lane < 32) reinterpret_cast<uint32_t *>(it.cdc_tail)[lane] = tl;
            }
        }
    };
    if (M == 0) {
        finish();
        return;
    }
    // twiddles and signs of this lane's transforms (position t) and of its
    // input-spectrum group (position lane_pos(kk))
    const PolLaneK<LPT> K(t, lane_pos(kk));

    // tap-digit spectra of this lane's filter and digit, N^-1 = -2048 folded in
    int32_t W[PPL];
    auto transform_taps = [&]() {
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            int32_t lo = ((w[j] + 64) & 127) - 64;
            int32_t hi = (w[j] - lo) >> 7;
            W[j] = td ? lo : hi;                      // |.| <= 64; W[NT..] is the padding
        }
        tap_fnt_lpt<LPT>(W, t, K);
    };
    transform_taps();

    const uint32_t nblocks = __builtin_amdgcn_readfirstlane((uint32_t)((M + 15) / 16));
    const int c2 = it.const_unit * it.const_unit;
    // 32-bit rounding shifts: |y| < 2^24 with out_shift <= 24; |G| <= 16 * 128 * 16
    // = 2^15, so every mu_shift above 17 rounds G to 0 exactly as 17 does
    const int out_s = it.out_shift;
    const int32_t out_r = out_s ? 1 << (out_s - 1) : 0;
    const int mu_early = __builtin_amdgcn_readfirstlane(min(it.mu_shift, 17));
    const int mu_late = __builtin_amdgcn_readfirstlane(min(it.mu_shift_late, 17));
    const int32_t mu_r_early = mu_early ? 1 << (mu_early - 1) : 0, mu_r_late = mu_late ? 1 << (mu_late - 1) : 0;
    // the step changes at block gear_at of this run (never: UINT32_MAX)
    const uint32_t gear_at = __builtin_amdgcn_readfirstlane(
        it.gear_blocks == 0u ? 0xFFFFFFFFu
                             : (it.block0 >= it.gear_blocks ? 0u
                                                            : (uint32_t)min<uint64_t>(it.gear_blocks - it.block0,
                                                                                      0xFFFFFFFFull)));
    bool bad = false;                                  // range violations, flagged once at the end
    // Windows: the lane holds window position wpos = (lane & 16) | lane_pos(lane &
    // 15), symbol 16 b - 16 + wpos of block b (the order the input-spectrum lanes
    // use, so a row swap hands every lane its two positions without LDS).  Window
    // loads are unconditional (index clamped into the input) and the zeros past
    // the end are applied when the window is used.
    const auto obase = gptr(it.out + 4 * om + 2 * pol + oS2l);
    const int wpos = (lane & 16) | lane_pos(lane & 15);
    src.prime();

    // Input spectra of the 4 streams of one block from its window (zeros past
    // the end applied): lane (S1 = lane / 16, k) writes positions kp, kp + 16 of
    // stream S1 to dst.
    auto spectra = [&](uint32_t win, int32_t(*dst)[kSpecRow]) {
        // rows 0, 2 hold positions lane_pos(l), rows 1, 3 positions 16 + lane_pos(l):
        // swapping odd rows of one copy with even rows of the other gives every
        // lane both (sw[0]: position kp, sw[1]: position kp + 16)
        const auto sw = __builtin_amdgcn_permlane16_swap(win, win, false, false);
        {
            const int kp = lane_pos(kk);                 // position index of this lane
            const int sh = 8 * (lane >> 4);              // byte of stream S1
            int32_t x0 = (int32_t)(int8_t)((uint32_t)sw[0] >> sh), x1 = (int32_t)(int8_t)((uint32_t)sw[1] >> sh);
            int32_t u0 = x0 + x1;
            int32_t u1 = fold16(opq((x0 - x1) << kp));   // |x0 - x1| <= 31: no overflow
            // lower lane u + p, upper lane (p - u) 2^e as one butterfly u a + p b
            // with (a, b) = (1, 1) or (-2^e, 2^e); u1 (|u1| < 2^16 + 15) keeps the
            // shift form at distance 8, where 2^e reaches 2^14
#pragma unroll
            for (int h = 8, hi = 0; h >= 2; h >>= 1, ++hi) {
                const int32_t a = K.spec[hi].a, b = K.spec[hi].b;    // xb_dif(kp, h)
                if (h == 8) {
                    const bool up = (kp & 8) != 0;
                    const int e = 2 * (kp & 7);              // <= 14
                    int32_t p1 = xor_pos<8>(u1);
                    u0 = xbfly<8>(u0, a, b);                // |u0| <= 32
                    u1 = blend(up, mul_pow2(p1 - u1, e), u1 + p1);
                } else {                                    // |u| < 2^17.01, 2^e <= 2^12
                    u0 = h == 4 ? xbfly<4>(u0, a, b) : xbfly<2>(u0, a, b);
                    u1 = h == 4 ? xbfly<4>(u1, a, b) : xbfly<2>(u1, a, b);
                }
            }
            // distance 1, twiddle 1
            u0 = xor_pos<1>(u0) + mul24k(u0, K.sgk);
            u1 = xor_pos<1>(u1) + mul24k(u1, K.sgk);
            dst[lane >> 4][kp] = u0;                    // |.| < 2^18
            dst[lane >> 4][kp + 16] = u1;
        }
    };

    // One block from its input spectra `spec` (position order, rows of kSpecRow
    // words by stream) and the window bytes `wbw` (rows of `row` bytes by
    // stream; the block's symbol 16 b at byte `woff` of each row).  `shadow` runs
    // in the shadow of the tap update's LDS reads, or in its place when the
    // update is off.
    auto block_core = [&](uint32_t b, const int32_t(*spec)[kSpecRow], const uint32_t *wbw, int row, int woff,
                          auto &&shadow) {
        // the step of this block (stream block block0 + b) under the schedule
        const int mu_s = b >= gear_at ? mu_late : mu_early;
        const int32_t mu_r = b >= gear_at ? mu_r_late : mu_r_early;
        const int64_t left = (int64_t)M - 16 * (int64_t)b;         // symbols from 16 b on
        int32_t Y[PPL];
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            int32_t P = mulmod(spec[tS1][t + LPT * j], W[j]);
            Y[j] = P + s1_partner<LPT>(P);              // pair sum over S1 = 2g, 2g+1
        }
        count_products(1, PPL);                         // A_S1 W for this lane's bins
        ifnt_upper_lpt<LPT>(Y, t, K);
        if (ts == 0) {
#pragma unroll
            for (int j = PPL / 2; j < PPL; ++j)
                part_h[b & 1][tg * 2 + td][(t + LPT * (j - PPL / 2)) * 2 + tS2l] = lift_loose(Y[j]);
        }
        if (WPP > 1) hsync.block(b); else wave_lds_sync();
        // symbol om, stream 2 pol + oS2l: y = 2^7 (high-digit sums) + (low-digit sums)
        const int pi = lane & 31;
        const int32_t(*part)[33] = part_h[b & 1];
        const int32_t y = 128 * (part[0][pi] + part[2][pi]) + part[1][pi] + part[3][pi];
        const int32_t yh = clamp32(rs32r(y, out_s, out_r), -32768, 32767);
        const bool valid = lane < 32 && om < left;
        if (writer && valid) obase[64 * (uint64_t)b] = (int16_t)yh;
        if (it.update_enable) {
            const int32_t yp = xor_h<1>(yh);
            const int64_t r2 = (int64_t)yh * yh + (int64_t)yp * yp;
            const int64_t R2 = r2 < 6LL * c2 ? 2LL * c2 : (r2 < 14LL * c2 ? 10LL * c2 : 18LL * c2);
            int32_t eps = (int32_t)clamp64(rs64((R2 - r2) * yh, it.err_shift), -128, 127);
            if (!valid) eps = 0;
            if (lane < 32) reinterpret_cast<int8_t *>(epsw)[oS2l * 16 + om] = (int8_t)eps;
            wave_lds_sync();
            // G[S1][S2][k] = sum_j eps_S2[j] * a_S1[16 b + j - k] for the lane's taps
            // k = t + LPT i: the 4 dwords of a_S1 from byte 16 b - k on.  Tap i's
            // dword q starts at byte base + 4 (q - S i) of the row, so the taps share
            // the aligned dwords j = q - S i in [J0, 3]: NJ byte alignments for the
            // NT * 4 dot products.
            constexpr int S = LPT / 4, J0 = -S * (NT - 1), NJ = 4 - J0;
            const int base = tS1 * row + woff - t;       // byte of a_S1[16 b - t]
            uint32_t e4[4], raw[NJ + 1];
#pragma unroll
            for (int q = 0; q < 4; ++q) e4[q] = epsw[tS2l * 4 + q];
#pragma unroll
            for (int r = 0; r <= NJ; ++r) raw[r] = wbw[(base >> 2) + J0 + r];
            shadow();                                    // in the shadow of the reads
            uint32_t ad[NJ];
#pragma unroll
            for (int r = 0; r < NJ; ++r) ad[r] = __builtin_amdgcn_alignbyte(raw[r + 1], raw[r], base & 3);
#pragma unroll
            for (int i = 0; i < NT; ++i) {
                int32_t gsum = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    gsum = __builtin_amdgcn_sdot4((int)e4[q], (int)ad[q - S * i - J0], gsum, false);
                w[i] = clamp32(w[i] + rs32r(gsum, mu_s, mu_r), -8192, 8191);   // step of this block
            }
            transform_taps();
        } else {
            shadow();
        }
        // the next block reuses this wave's window and error bytes: keep the LDS
        // reads above in front of the writes that follow
        wave_lds_sync();
    };

    if constexpr (Src::kSegmented) {
        // The window of block b + 2 is loaded during block b into the register
        // block b's came in (even and odd blocks alternate between two); block b
        // computes block b + 1's input spectra into the other of two buffers while
        // it waits for the LDS reads of its tap update, off the chain from one
        // block's taps to the next.  Window bytes: rows of 32 (+ 4 zero) bytes.
        if (lane < 4) winw[32 + lane] = 0u;
        auto block = [&](uint32_t b, uint32_t &win, uint32_t win_next) {
            const int64_t left = (int64_t)M - 16 * (int64_t)b;
            if (wpos - 16 >= left) win = 0u;                        // past the end
            bad |= !bytes_5bit(win);
            if (lane < 32) {       // window bytes by stream for the tap update
                uint8_t *wb = reinterpret_cast<uint8_t *>(winw);
#pragma unroll
                for (int c = 0; c < 4; ++c) wb[c * 32 + wpos] = (uint8_t)(win >> (8 * c));
            }
            win = src.ahead(b, wpos);                               // symbol 16 b + 16 + wpos
            // block b + 1's window position wpos is symbol 16 b + wpos
            const uint32_t wn = wpos >= left ? 0u : win_next;
            block_core(b, aspec[b & 1], winw, 32, 16, [&] { spectra(wn, aspec[(b + 1) & 1]); });
        };
        uint32_t win_even = src.first(-16 + wpos), win_odd = src.first(wpos);   // blocks 0 and 1
        spectra(wpos - 16 >= (int64_t)M ? 0u : win_even, aspec[0]);
        wave_lds_sync();
        // segments of 64 blocks (an even count keeps each block's window register)
        for (uint32_t b0 = 0; b0 < nblocks; b0 += 64) {
            const uint32_t b1 = min(b0 + 64u, nblocks);
            src.segment(b0, b1);
            for (uint32_t b = b0; b < b1; b += 2) {
                block(b, win_even, win_odd);
                if (b + 1 < b1) block(b + 1, win_odd, win_even);
            }
            src.segment_done(b1);
        }
    } else {
        // Batches of kBatch blocks.  A batch's 144 window symbols (16 b0 - 16 ..
        // 16 b0 + 127, history before 0, zeros past M) are fetched one batch
        // ahead, three per lane, and staged as bytes by stream (rows of kStgRow
        // bytes, the tail zero); the input spectra of its 4 streams x kBatch
        // blocks are then the matrix product of Eq. (1)'s transform matrix (rows
        // in position order, bin bitrev5(p) at position p) with the 32-symbol
        // windows, on the matrix cores in 8-bit digits: each entry 2^(nk) mod F
        // is a signed power of two, written as 256 hi + lo with int8 hi, lo
        // (2^15 as -32769 = 256 (-128) - 1, congruent modulo F).  Four
        // v_mfma_i32_32x32x16_i8: hi digits over positions 0-15 and 16-31, the
        // accumulator times 256, then lo.  |sum| <= 32 * 128 * 16 (257) < 2^24.1,
        // one fold, |X| < 2^17.
        uint8_t *const stgb = reinterpret_cast<uint8_t *>(winw);
        if (lane < 16) winw[(lane >> 2) * (kStgRow / 4) + 36 + (lane & 3)] = 0u;   // row tails: bytes 144..159
        // operand lanes of v_mfma_i32_32x32x16_i8: lane l holds row (A) or column (B)
        // l % 32 and the 8 K indices 8 (l / 32) + e of its 16-wide K slice
        const int mp = lane & 31, mkb = bitrev5(mp), mnh = 8 * (lane >> 5);
        uint64_t a_hi[2], a_lo[2];
#pragma unroll
        for (int kh = 0; kh < 2; ++kh) {
            uint64_t hi = 0, lo = 0;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int m = (mkb * (16 * kh + mnh + e)) & 31;
                const int pw = m & 15, neg = m & 16;
                int dh, dl;
                if (pw <= 6) { dh = 0; dl = neg ? -(1 << pw) : (1 << pw); }
                else if (pw == 7) { dh = neg ? 0 : 1; dl = -128; }
                else if (pw <= 14) { dh = neg ? -(1 << (pw - 8)) : (1 << (pw - 8)); dl = 0; }
                else { dh = -128; dl = neg ? 0 : -1; }
                hi |= (uint64_t)(uint8_t)dh << (8 * e);
                lo |= (uint64_t)(uint8_t)dl << (8 * e);
            }
            a_hi[kh] = hi;
            a_lo[kh] = lo;
        }
        const auto a32 = src.base;
        const auto h32 = gptr(reinterpret_cast<const uint32_t *>(it.hist_in));
        uint32_t pre[3];
        auto fetch = [&](uint32_t b0) {
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int q = lane + 64 * r;
                const int64_t i = 16 * (int64_t)b0 - 16 + q;
                uint32_t v = 0u;
                if (q < 144) {
                    if (i < 0) {
                        if (it.hist_in != nullptr) v = h32[16 + i];
                    } else if ((uint64_t)i < M) {
                        v = a32[i];
                    }
                }
                pre[r] = v;
            }
        };
        fetch(0);
        const int mj = lane & 31, mjb = mj >> 2, ms = mj & 3;   // this lane's column: block mjb, stream ms
        for (uint32_t b0 = 0; b0 < nblocks; b0 += kBatch) {
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int q = lane + 64 * r;
                if (q < 144) {
                    const uint32_t v = pre[r];
                    bad |= !bytes_5bit(v);
#pragma unroll
                    for (int c = 0; c < 4; ++c) stgb[c * kStgRow + q] = (uint8_t)(v >> (8 * c));
                }
            }
            fetch(b0 + kBatch);                          // the next batch
            wave_lds_sync();
            const uint8_t *col = stgb + ms * kStgRow + 16 * mjb + mnh;
            const int64_t bx0 = (int64_t)*reinterpret_cast<const uint64_t *>(col);
            const int64_t bx1 = (int64_t)*reinterpret_cast<const uint64_t *>(col + 16);
            v16i acc = {};
            acc = __builtin_amdgcn_mfma_i32_32x32x16_i8((int64_t)a_hi[0], bx0, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_i32_32x32x16_i8((int64_t)a_hi[1], bx1, acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = (int32_t)((uint32_t)acc[r] << 8);
            acc = __builtin_amdgcn_mfma_i32_32x32x16_i8((int64_t)a_lo[0], bx0, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_i32_32x32x16_i8((int64_t)a_lo[1], bx1, acc, 0, 0, 0);
            // lane: column (mjb, ms), register r: position 8 (r / 4) + 4 (lane / 32) + r % 4
#pragma unroll
            for (int g = 0; g < 4; ++g)
                *reinterpret_cast<int4 *>(&aspec[mjb][ms][8 * g + 4 * (lane >> 5)]) =
                    make_int4(fold16(acc[4 * g]), fold16(acc[4 * g + 1]), fold16(acc[4 * g + 2]),
                              fold16(acc[4 * g + 3]));
            wave_lds_sync();
            const uint32_t nb = min((uint32_t)kBatch, nblocks - b0);
            for (uint32_t jb = 0; jb < nb; ++jb)
                block_core(b0 + jb, aspec[jb], winw, kStgRow, 16 * (int)jb + 16, [] {});
        }
    }
    if (bad) flag(err, RANGE_SYMBOL);
    finish();
}

// IW = 1: one half per workgroup, the halves paired on XCDs as above.  IW = 2
// (one wave per half only): both halves of a channel in one workgroup of two
// independent waves (wave v runs polarisation v), one workgroup per channel.
template <int LPT, int IW = 1>
__device__ __forceinline__ void aeq_pol_body(const AeqItem *items, int n, const AeqItem &single, int *err,
                                             int prio, unsigned bid) {
    static_assert(IW == 1 || (IW == 2 && LPT == 4), "paired halves need one wave per half");
    const unsigned ch = IW == 1 ? (bid >> 4) * 8 + (bid & 7) : bid;
    if (ch >= (unsigned)(items ? n : 1)) return;       // padding of the last run of 16
    // latency-critical chains (the longest of a batch) issue ahead of the
    // throughput work that shares their SIMDs
    if (prio) __builtin_amdgcn_s_setprio(3);
    constexpr int WPP = LPT / 4;                       // waves per polarisation half
    const AeqItem it = items ? items[ch] : single;
    const int tid = threadIdx.x;
    const int v = tid >> 6, lane = tid & 63;
    const int vh = v % WPP;                            // wave within its half
    const int pol = IW == 1 ? (int)((bid >> 3) & 1) : v;

    // spectra rows of 36 words: the products' lanes reading one position of the
    // 4 rows (and 4 positions apart) hit 16 different banks
    __shared__ __align__(16) int32_t aspec_s[WPP * IW][kBatch][4][kSpecRow];   // per wave: a batch's input spectra
    // per half: [block parity][g*2+d][m*2+S2l], shared by the half's waves;
    // double-buffered so a wave that runs ahead (one barrier per block) never
    // overwrites partials another wave is still reading
    __shared__ int32_t part_s[IW][2][4][33];
    __shared__ uint32_t epsw_s[WPP * IW][8];           // per wave: bytes [S2l][m]
    __shared__ __align__(16) uint32_t winw_s[WPP * IW][kStgRow];   // per wave: a batch's window bytes [S1][kStgRow]
    AeqSrcGlobal src{&it, gptr(reinterpret_cast<const uint32_t *>(it.a)), it.m};
    HalfSyncWg hs;
    aeq_pol_run<LPT>(it, pol, vh, lane, err, aspec_s[v], part_s[v / WPP], epsw_s[v], winw_s[v], src, hs);
}

template <int LPT, int IW = 1>
__global__ __launch_bounds__(64 * (LPT / 4) * IW) void aeq_pol_kernel(const AeqItem *items, int n,
                                                                      AeqItem single, int *err, int prio) {
    aeq_pol_body<LPT, IW>(items, n, single, err, prio, blockIdx.x);
}

// ------------------------------------------------------------------------
// Fused persistent FNT-CDC + FNT-AEQ (the receiver chain of the experimental
// section: CDC, resampling to 1 sample/symbol, AEQ) in one launch.
//
// A workgroup runs one channel at a time: 2 WPP consumer waves run the two
// polarisation halves of the AEQ (aeq_pol_run), and NP producer waves run the
// lane-per-block CDC (cdc_lane_blocks) 64 blocks (one chunk) at a time into a
// ring of RING chunks in LDS, producer p taking the chunks c = p mod NP (so
// that the CDC spreads over the SIMDs the consumers run on).  The
// 1-sample/symbol stream never leaves the CU.  Hand-offs, all in LDS:
//   * slots[s]: 1 + the chunk slot s holds, written after the chunk; a consumer
//     loading the window of block b + 2 needs chunk min(16 b + 47, M - 1) / 1024;
//   * cons[v]: blocks finished by consumer wave v, published after every
//     segment of 64 blocks (the chunks a segment reads ahead are checked once,
//     before it); after block b a wave never reads a symbol below
//     16 (b + 1) + 16 again, so a producer may rewrite the slot of chunk
//     c - RING once every wave has published 64 (c - RING + 1) - 1 blocks.
// Neither side waits for more than the other can supply with RING >= 4 chunks,
// so the waits end; each also gives up after a bound (RANGE_STALL).  Channels
// come from a work counter (queue[0]) in table order (longest chains first), so
// the longest chains start at once on the first workgroups and the others fill
// in as workgroups free up; the last workgroup to find the table empty resets
// the counters (queue[0], queue[1]) for the next launch.  Without a counter
// (queue = nullptr) workgroup w runs channel w once.  Channels with index <
// nprio run at raised wave priority (the producers one level below their
// consumers: they run up to RING chunks ahead and only have to keep ahead).
// ------------------------------------------------------------------------
// HALVES = 2: a workgroup runs both halves of its channel (2 WPP consumer
// waves, one producer set); HALVES = 1: a workgroup runs one half and has its
// own producers (the CDC is computed once per half), the halves of a channel
// in the two workgroups of a pair 8 indices apart (one XCD, as for the plain
// polarisation-split AEQ), for the shortest serial latency when the GPU is
// otherwise idle.  HALVES = 1 takes no work counter.
template <int LPT, int NP, int HALVES>
__global__ __launch_bounds__(64 * (HALVES * (LPT / 4) + NP)) __attribute__((amdgpu_waves_per_eu(3))) void cdc_aeq_fused_kernel(
    const CdcItem *__restrict__ citems, const AeqItem *__restrict__ aitems, int n, CdcItem csingle, AeqItem asingle,
    uint32_t *queue, int nprio, int *err, uint32_t spin_limit) {
    constexpr int WPP = LPT / 4;
    constexpr int NC = HALVES * WPP;                   // consumer waves
    constexpr int RING = NP >= 4 ? 8 : 4;              // a power of two, >= 2 NP
    static_assert(NP == 1 || NP == 2 || NP == 4, "producer waves");
    static_assert(HALVES == 1 || HALVES == 2, "halves per workgroup");
    const int v = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // HALVES = 1: workgroup bid runs half (bid >> 3) & 1 of channel (bid >> 4) * 8 + (bid & 7)
    const unsigned bid = blockIdx.x;
    const int my_pol = HALVES == 1 ? (int)((bid >> 3) & 1) : 0;
    const unsigned my_ch = HALVES == 1 ? (bid >> 4) * 8 + (bid & 7) : bid;


    __shared__ __align__(16) uint32_t ring_s[RING * FUSED_CHUNK_SYMS];
    __shared__ uint32_t slot_s[RING], cons_s[NC], next_s, stall_s;
    __shared__ __align__(16) uint32_t arrive_s[HALVES][WPP < 2 ? 2 : WPP];
    __shared__ int32_t hs_s[NP][2][64];
    __shared__ __align__(16) uint32_t edge_s[NP][2][64];
    __shared__ int32_t aspec_s[NC][2][4][kSpecRow];
    __shared__ int32_t part_s[HALVES][2][4][33];
    __shared__ uint32_t epsw_s[NC][8];
    __shared__ uint32_t winw_s[NC][36];

    const int total = citems ? n : 1;
    // Both roles run the same sequence of workgroup barriers, two per channel,
    // in loops of their own (so that neither role's loop-invariant lane
    // constants stay live through the other role's code).  Thread 0 (consumer
    // wave 0) takes the next channel; consumer wave 0 clears the hand-off words.
    auto next_channel = [&](uint32_t iter) -> uint32_t {
        if (threadIdx.x == 0) {
            // with a work counter: the next channel of the table; without: channel
            // blockIdx.x, once
            next_s = queue ? atomicAdd(&queue[0], 1u) : (iter == 0 ? my_ch : 0xFFFFFFFFu);
            if (iter == 0) stall_s = 0;
        }
        if (threadIdx.x < NC) {
            cons_s[threadIdx.x] = 0;
            arrive_s[threadIdx.x / WPP][threadIdx.x % WPP] = 0;
        }
        if (threadIdx.x < RING) slot_s[threadIdx.x] = 0;
        __syncthreads();
        // the same for every lane: the channel's item and all that follows from it
        // stay in scalar registers and branch uniformly
        return __builtin_amdgcn_readfirstlane(next_s);
    };
    if (v >= NC) {                                     // producers: the CDC of each channel
        const int pv = v - NC;
        for (uint32_t iter = 0;; ++iter) {
            const uint32_t chn = next_channel(iter);
            if (chn >= (uint32_t)total) break;
            if ((int)chn < nprio) __builtin_amdgcn_s_setprio(2); else __builtin_amdgcn_s_setprio(0);
            const CdcItem *ip = citems ? &citems[chn] : &csingle;
            const uint64_t nb = fnti::cdc_blocks(ip->n);
            const uint32_t nchunks = (uint32_t)((nb + fnti::CDC_CHUNK - 1) / fnti::CDC_CHUNK);
            cdc_lane_spectra(ip, lane, hs_s[pv]);
            wave_lds_sync();
            bool live = true;
            for (uint32_t c = pv; c < nchunks; c += NP) {
                if (c >= (uint32_t)RING && live) {     // slot of chunk c - RING free?
                    const uint32_t need = (uint32_t)fnti::CDC_CHUNK * (c - RING + 1) - 1;
#pragma unroll
                    for (int k = 0; k < NC; ++k)
                        if (live) live = wait_at_least<32>(&cons_s[k], need, spin_limit, err, &stall_s);
                }
                uint32_t o[16];
                cdc_lane_blocks(ip, (uint64_t)c * fnti::CDC_CHUNK, lane, hs_s[pv], edge_s[pv], err, o,
                                reinterpret_cast<uint16_t *>(&ring_s[(c % RING) * FUSED_CHUNK_SYMS]));
                if (lane == 0) lds_store_rel(&slot_s[c % RING], c + 1);   // after the wave's ring writes
                wave_lds_sync();
            }
            __syncthreads();                           // the channel is done; LDS is free again
        }
    } else {                                           // consumers: the AEQ halves of each channel
        const int pol = HALVES == 2 ? v / WPP : my_pol, vh = v % WPP;
        for (uint32_t iter = 0;; ++iter) {
            const uint32_t chn = next_channel(iter);
            if (chn >= (uint32_t)total) break;
            if ((int)chn < nprio) __builtin_amdgcn_s_setprio(3); else __builtin_amdgcn_s_setprio(1);
            const AeqItem it = aitems ? aitems[chn] : asingle;
            AeqSrcRing<RING> src{&it, ring_s, slot_s, &cons_s[v], &stall_s, it.m, spin_limit, err, 0u, true,
                                 HALVES == 2 ? &cons_s[(1 - pol) * WPP] : nullptr, HALVES == 2 ? WPP : 0};
            if constexpr (WPP == 1) {
                HalfSyncWg unused;
                aeq_pol_run<LPT>(it, pol, vh, lane, err, aspec_s[v], part_s[v / WPP], epsw_s[v], winw_s[v], src,
                                 unused);
            } else {
                HalfSyncLds<WPP> hsync{arrive_s[v / WPP], &stall_s, spin_limit, err, vh, true};
                aeq_pol_run<LPT>(it, pol, vh, lane, err, aspec_s[v], part_s[v / WPP], epsw_s[v], winw_s[v], src,
                                 hsync);
            }
            __syncthreads();                           // the channel is done; LDS is free again
        }
    }
    if (queue && threadIdx.x == 0) {                   // the last workgroup out resets the counters
        if (atomicAdd(&queue[1], 1u) == gridDim.x - 1) {
            __hip_atomic_store(&queue[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&queue[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ------------------------------------------------------------------------
// FNT-AEQ, one whole transform per lane (throughput form).
//
// A wave runs two channels, one per 32-lane slot.  Lane t of a slot owns the
// tap filter f = t / 2 (S1 = f / 4, S2 = f % 4) and digit d = t % 2 (0: the
// high 7-bit digit, 1: the low one): its 32-bin tap-digit spectrum W stays in
// its registers and every transform it needs runs in its registers, with no
// exchange between lanes inside a transform.  Per 16-symbol block:
//   * the input spectra A_S1 come from LDS, computed eight blocks ahead, one
//     transform per lane (stream S1 = t % 4, block t / 4 of the batch);
//   * P = A_S1 W; lanes t and t ^ 8 (S1 = 2g, 2g + 1) sum their products (the
//     Eq. (5) bound of the balanced digits holds for the pair), and the lanes
//     with S1 even invert the sum (upper half of the 32-point inverse);
//   * y_S2 = 2^7 (high-digit sums) + (low-digit sums): lanes t ^ 1 (digits) and
//     t ^ 16 (pairs) add up, and the S2 lanes hand the 16 outputs over LDS to
//     the output / error lanes (symbol t / 2, polarisation t % 2);
//   * the RDE gradient of Eq. (6) for the lane's 8 taps by 4-byte dot products
//     over the staged input bytes, the tap update, the other 8 taps from the
//     digit partner t ^ 1, and the new digit spectrum.
// ------------------------------------------------------------------------

// (a - b) * 2^E for a compile-time E in [0, 16).
template <int E>
__device__ __forceinline__ int32_t tw2_diff(int32_t a, int32_t b) {
    if constexpr (E == 0) return a - b;
    else if constexpr (E < 15) return mul_pow2(a - b, E);
    else return mulmod(a - b, opq(32768));
}

// 32-point DIF forward transform (radix 2) in registers, natural order in,
// x[n] = bin bitrev5(n) out.  ZP: inputs 16..31 are zero.
// In: |x| <= 2^17; out: |X| < 2^21.1.
template <int H>
__device__ __forceinline__ void fnt32_stage(int32_t (&x)[32]) {
    sfor<16 / H>([&](auto gc) {
        constexpr int g = decltype(gc)::value * 2 * H;
        sfor<H>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const int32_t a = x[g + j], b = x[g + j + H];
            x[g + j] = a + b;
            x[g + j + H] = tw2_diff<j * (16 / H)>(a, b);
        });
    });
}
template <bool ZP>
__device__ __forceinline__ void fnt32_regs(int32_t (&x)[32]) {
    if constexpr (ZP) {
        sfor<16>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            x[j + 16] = tw2_diff<j>(x[j], 0);
        });
    } else {
        fnt32_stage<16>(x);
    }
    fnt32_stage<8>(x);
    fnt32_stage<4>(x);
    fnt32_stage<2>(x);
    fnt32_stage<1>(x);
}

template <int WPG>
__device__ __forceinline__ void aeq_lane_body(const AeqItem *items, int nitems, const AeqItem &single,
                                              int *err, int prio, unsigned bid) {
    if (prio) __builtin_amdgcn_s_setprio(3);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int slot = lane >> 5, t = lane & 31;
    const int item = ((int)bid * WPG + wv) * 2 + slot;
    const bool has = items ? item < nitems : item == 0;
    // LDS of this wave, by slot
    __shared__ __align__(16) int32_t aspec_s[WPG][2][8][4][32];   // input spectra [block of batch][S1][bin]
    __shared__ __align__(16) uint32_t abytes_s[WPG][2][4][40];    // staged input bytes [S1][160]
    __shared__ __align__(16) int32_t ybuf_s[WPG][2][4][16];       // outputs y [S2][symbol]
    __shared__ __align__(16) uint32_t eps_s[WPG][2][4][4];        // RDE errors, bytes [S2][symbol]
    int32_t(*aspec)[4][32] = aspec_s[wv][slot];
    uint32_t(*abytes)[40] = abytes_s[wv][slot];
    int32_t(*ybuf)[16] = ybuf_s[wv][slot];
    uint32_t(*epsw)[4] = eps_s[wv][slot];

    const AeqItem *ip = items ? &items[has ? item : 0] : &single;
    const uint64_t M = has ? ip->m : 0;
    const int8_t *ain = ip->a;
    const int8_t *hist_in = ip->hist_in;
    int16_t *outp = ip->out;
    int16_t *taps = ip->taps;
    // rs(G, s) of a gradient |G| <= 32768 is 0 for every s >= 17, so a shift
    // clamped to 20 gives the same result in 32-bit arithmetic
    const int out_shift = ip->out_shift, err_shift = ip->err_shift;
    const int mu_early = ip->mu_shift < 20 ? ip->mu_shift : 20;
    const int mu_late = ip->mu_shift_late < 20 ? ip->mu_shift_late : 20;
    const uint32_t gear = ip->gear_blocks;
    const uint64_t blk0 = ip->block0;
    const int64_t c2 = (int64_t)ip->const_unit * ip->const_unit;
    const bool upd = has && ip->update_enable != 0;
    const uint32_t nb = (uint32_t)((M + 15) / 16);
    const uint32_t nbw = max((uint32_t)__shfl((int)nb, 0), (uint32_t)__shfl((int)nb, 32));

    // tap role
    const int f = t >> 1, d = t & 1;
    const int S1 = f >> 2, S2 = f & 3;
    int32_t w[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        int32_t val = has ? taps[f * 16 + k] : 0;
        if (val < -8192 || val > 8191) flag(err, RANGE_TAP);
        w[k] = clamp32(val, -8192, 8191);
    }
    auto finish = [&]() {                              // the slot's channel is done
        if (!has) return;
#pragma unroll
        for (int i = 0; i < 8; ++i) taps[f * 16 + 8 * d + i] = (int16_t)(d ? w[8 + i] : w[i]);
        if (ip->hist_out) {
            uint32_t h = 0u;
            if (t < 16) {
                const int64_t i = (int64_t)M - 16 + t;
                if (i >= 0) h = reinterpret_cast<const uint32_t *>(ain)[i];
                else if (hist_in) h = reinterpret_cast<const uint32_t *>(hist_in)[16 + i];
            }
            if (t < 16) reinterpret_cast<uint32_t *>(ip->hist_out)[t] = h;
        }
        if (ip->cdc_tail) {
            const int64_t j = (int64_t)ip->cdc_n - 32 + t;
            const uint32_t tl = j >= 0 ? reinterpret_cast<const uint32_t *>(ip->cdc_in)[j]
                                       : reinterpret_cast<const uint32_t *>(ip->cdc_tail)[32 + j];
            reinterpret_cast<uint32_t *>(ip->cdc_tail)[t] = tl;
        }
    };
    if (M == 0) finish();
    if (nbw == 0) return;

    // tap-digit spectrum of this lane, N^-1 = 32^-1 = -2048 folded in
    int32_t W[32];
    // digits w = 2^7 hi + lo, hi = (w + 64) >> 7 in [-64, 64], lo in [-64, 63]:
    // digit d times -2048 is w A + hi B with A = 0, B = -2048 (d = 0) or
    // A = -2048, B = 2^18 (d = 1), one 24-bit multiply-add per tap
    const int32_t dA = d ? -2048 : 0, dB = d ? 262144 : -2048;
    auto transform_taps = [&]() {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int32_t hi = (w[k] + 64) >> 7;
            W[k] = sext24(w[k]) * dA + sext24(hi) * dB;      // |.| <= 2^17
            W[k + 16] = 0;
        }
        fnt32_regs<true>(W);
    };
    transform_taps();
    if (t < 4) abytes[t][36] = abytes[t][37] = abytes[t][38] = abytes[t][39] = 0u;
    uint32_t bad = 0u;
    const int om = t >> 1, opol = t & 1;                // output / error role

    for (uint32_t b = 0; b < nbw; ++b) {
        const int mu_shift = (gear != 0u && blk0 + b >= (uint64_t)gear) ? mu_late : mu_early;   // step schedule
        const int j = (int)(b & 7);
        if (j == 0) {
            // stage symbols 16 b - 16 .. 16 b + 127 of the four streams as bytes
            // (global-address loads: a generic one would make every LDS wait of
            // the loop wait for memory too)
            wave_lds_sync();
#pragma unroll
            for (int r = 0; r < 5; ++r) {
                const int p = t + 32 * r;
                if (p < 144) {
                    const int64_t i = 16 * (int64_t)b - 16 + p;
                    uint32_t v = 0u;
                    if (i < 0) {
                        if (hist_in) v = gptr(reinterpret_cast<const uint32_t *>(hist_in))[16 + i];
                    } else if ((uint64_t)i < M) {
                        v = gptr(reinterpret_cast<const uint32_t *>(ain))[i];
                        bad |= v ^ (v << 1);
                    }
                    uint8_t *ab = reinterpret_cast<uint8_t *>(&abytes[0][0]);
#pragma unroll
                    for (int c = 0; c < 4; ++c) ab[c * 160 + p] = (uint8_t)(v >> (8 * c));
                }
            }
            wave_lds_sync();
            {   // input spectra of the batch: stream t % 4, block t / 4
                const int s1 = t & 3, jb = t >> 2;
                const uint4 *src = reinterpret_cast<const uint4 *>(&abytes[s1][4 * jb]);
                int32_t x[32];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const uint4 v4 = src[q];
                    const uint32_t vv[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
                    for (int c = 0; c < 4; ++c)
#pragma unroll
                        for (int e = 0; e < 4; ++e) x[16 * q + 4 * c + e] = sbyte(vv[c], e);
                }
                fnt32_regs<false>(x);
                int4 *dst = reinterpret_cast<int4 *>(&aspec[jb][s1][0]);
#pragma unroll
                for (int q = 0; q < 8; ++q) dst[q] = make_int4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
            }
            wave_lds_sync();
        }
        const bool live = b < nb;
        // products, pair sums over S1 = 2g, 2g + 1, and the inverse
        int32_t Y[32];
        {
            const int4 *A4 = reinterpret_cast<const int4 *>(&aspec[j][S1][0]);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int4 a4 = A4[q];
                Y[4 * q] = mulmod(a4.x, W[4 * q]);
                Y[4 * q + 1] = mulmod(a4.y, W[4 * q + 1]);
                Y[4 * q + 2] = mulmod(a4.z, W[4 * q + 2]);
                Y[4 * q + 3] = mulmod(a4.w, W[4 * q + 3]);
            }
        }
#pragma unroll
        for (int k = 0; k < 32; ++k) Y[k] += xor_lane<8>(Y[k]);   // |.| < 2^17.4
        ifnt32_upper_regs(Y);
        // y_S2 = 2^7 (hi sums) + (lo sums): digits from t ^ 1, pairs from t ^ 16
        int32_t yv[16];
        const int32_t dscale = d ? 1 : 128;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            int32_t v = sext24(lift_z(Y[16 + q])) * dscale;
            v += xor_lane<1>(v);
            v += xor_lane<16>(v);
            yv[q] = v;                                  // |.| < 2^23.1
        }
        if (t < 8 && d == 0) {                          // lanes of g = 0, digit 0: S2 = t / 2
            int4 *yd4 = reinterpret_cast<int4 *>(&ybuf[S2][0]);
#pragma unroll
            for (int q = 0; q < 4; ++q) yd4[q] = make_int4(yv[4 * q], yv[4 * q + 1], yv[4 * q + 2], yv[4 * q + 3]);
        }
        wave_lds_sync();
        // outputs and RDE errors: symbol om, streams 2 opol (I), 2 opol + 1 (Q)
        const int64_t m = 16 * (int64_t)b + om;
        const bool valid = live && (uint64_t)m < M;
        const int32_t yi = ybuf[2 * opol][om], yq = ybuf[2 * opol + 1][om];
        const int32_t hi_ = clamp32((yi + ((1 << out_shift) >> 1)) >> out_shift, -32768, 32767);
        const int32_t hq_ = clamp32((yq + ((1 << out_shift) >> 1)) >> out_shift, -32768, 32767);
        if (valid)
            gptr(reinterpret_cast<uint32_t *>(outp))[2 * m + opol] = ((uint32_t)hi_ & 0xFFFFu) | ((uint32_t)hq_ << 16);
        if (__ballot(upd && live)) {
            const int64_t r2 = (int64_t)hi_ * hi_ + (int64_t)hq_ * hq_;
            const int64_t R2 = r2 < 6 * c2 ? 2 * c2 : (r2 < 14 * c2 ? 10 * c2 : 18 * c2);
            int32_t ei = (int32_t)clamp64(rs64((R2 - r2) * hi_, err_shift), -128, 127);
            int32_t eq = (int32_t)clamp64(rs64((R2 - r2) * hq_, err_shift), -128, 127);
            if (!valid) ei = eq = 0;
            uint8_t *eb = reinterpret_cast<uint8_t *>(&epsw[0][0]);
            eb[(2 * opol) * 16 + om] = (uint8_t)ei;
            eb[(2 * opol + 1) * 16 + om] = (uint8_t)eq;
            wave_lds_sync();
            // G[k] = sum_m eps_S2[m] a_S1[16 b + m - k] for k = 8 d + i (i < 8)
            uint32_t e4[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) e4[q] = epsw[S2][q];
            uint32_t dd[7];
            const int q0 = 4 * j + 2 - 2 * d;            // byte 4 q0 = 16 j + 8 - 8 d
#pragma unroll
            for (int r = 0; r < 7; ++r) dd[r] = abytes[S1][q0 + r];
            int32_t g[8];
            sfor<8>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int o = 8 - i;                    // a_S1[16 b - k] is byte o of dd
                int32_t gs = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    gs = __builtin_amdgcn_sdot4((int)e4[q],
                                                (int)__builtin_amdgcn_alignbyte(dd[(o >> 2) + q + 1],
                                                                                dd[(o >> 2) + q], o & 3),
                                                gs, false);
                g[i] = gs;                                  // |.| <= 32768
            });
            const bool step = upd && live;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int32_t mine = d ? opq(w[8 + i]) : opq(w[i]);
                const int32_t nw = clamp32(mine + ((g[i] + ((1 << mu_shift) >> 1)) >> mu_shift), -8192, 8191);
                const int32_t upd_w = step ? nw : mine;
                const int32_t other = xor_lane<1>(upd_w);   // the digit partner's taps 8 (1 - d) + i
                w[i] = d ? other : upd_w;
                w[8 + i] = d ? upd_w : other;
            }
            transform_taps();
            // the next block rewrites the error bytes: keep the reads above in front
            wave_lds_sync();
        }
        if (live && b + 1 == nb) finish();
    }
    if ((bad & 0xE0E0E0E0u) != 0u) flag(err, RANGE_SYMBOL);
}

template <int WPG>
__global__ __launch_bounds__(64 * WPG) void aeq_lane_kernel(const AeqItem *items, int nitems,
                                                            AeqItem single, int *err, int prio) {
    aeq_lane_body<WPG>(items, nitems, single, err, prio, blockIdx.x);
}

// ------------------------------------------------------------------------
// FNT-AEQ, one channel per wave, two lanes per transform (latency + throughput).
//
// Lane L plays role L: bit 0 = half h of the 32 bins (positions 16 h + j, j < 16,
// in registers), bit 1 = digit d, bit 2 = g and bit 3 = s of S1 = 2 g + s,
// bits 4-5 = S2.  Only the first stage of the forward transform and the last
// stage of the inverse cross the two halves; both lanes of a transform hold all
// 16 taps, so the forward one needs no exchange at all (the upper half is the
// zero-padded half: its first-stage value is digit * 2^j).  Partners: pair sum
// over s (lanes L ^ 8, DPP row_ror:8), digit sum (L ^ 2, quad_perm), group sum
// over g (L ^ 4, swizzle), inverse halves (L ^ 1, quad_perm); the four lanes of
// a filter (L ^ 0..3) share its taps by quad broadcasts.
// ------------------------------------------------------------------------

// Radix-2 stages of the 32-point forward (DIF) / inverse (DIT) transforms on
// N consecutive positions held in registers (N = 16: one half).
template <int H, int N>
__device__ __forceinline__ void fwd_stage_n(int32_t (&x)[N]) {
    sfor<N / (2 * H)>([&](auto gc) {
        constexpr int g = decltype(gc)::value * 2 * H;
        sfor<H>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const int32_t a = x[g + j], b = x[g + j + H];
            x[g + j] = a + b;
            x[g + j + H] = tw2_diff<j * (16 / H)>(a, b);
        });
    });
}
template <int H, int N>
__device__ __forceinline__ void inv_stage_n(int32_t (&y)[N]) {
    sfor<N / (2 * H)>([&](auto gc) {
        constexpr int g = decltype(gc)::value * 2 * H;
        sfor<H>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            int32_t lo, hi;
            inv_bfly<j * (16 / H)>(y[g + j], y[g + j + H], lo, hi);
            y[g + j] = lo;
            y[g + j + H] = hi;
        });
    });
}

// -b 2^-E (mod 65537) for a compile-time E in [0, 16): 2^-E = -2^(16 - E).
template <int E>
__device__ __forceinline__ int32_t neg_inv_tw(int32_t b) {
    if constexpr (E == 0) return -b;
    else if constexpr (E == 1) return mulmod(b, opq(32768));
    else return mul_pow2(b, 16 - E);
}

// Value of lane (L & ~3) | Q of the lane's quad.
template <int Q>
__device__ __forceinline__ int32_t quad_bcast(int32_t v) {
    return __builtin_amdgcn_update_dpp(0, v, Q * 0x55, 0xF, 0xF, true);
}

template <int WPG>
__device__ __forceinline__ void aeq_duo_body(const AeqItem *items, int nitems, const AeqItem &single,
                                             int *err, int prio, unsigned bid) {
    if (prio) __builtin_amdgcn_s_setprio(3);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int item = (int)bid * WPG + wv;
    if (items ? item >= nitems : item != 0) return;
    const AeqItem *ip = items ? &items[item] : &single;
    const int hh = lane & 1, d = (lane >> 1) & 1, gs = (lane >> 2) & 1, ss = (lane >> 3) & 1;
    const int S1 = 2 * gs + ss, S2 = lane >> 4;
    const int f = S1 * 4 + S2, qd = lane & 3;           // filter, position in the filter's quad
    __shared__ __align__(16) int32_t aspec_s[WPG][16][4][32];   // input spectra of 16 blocks
    __shared__ __align__(16) uint32_t abytes_s[WPG][4][72];     // staged input bytes [S1][288]
    __shared__ __align__(16) int32_t ybuf_s[WPG][4][16];        // outputs y [S2][symbol]
    __shared__ __align__(16) uint32_t eps_s[WPG][4][4];         // RDE errors, bytes [S2][symbol]
    int32_t(*aspec)[4][32] = aspec_s[wv];
    uint32_t(*abytes)[72] = abytes_s[wv];
    int32_t(*ybuf)[16] = ybuf_s[wv];
    uint32_t(*epsw)[4] = eps_s[wv];

    const uint64_t M = ip->m;
    const int8_t *ain = ip->a;
    const int8_t *hist_in = ip->hist_in;
    int16_t *outp = ip->out;
    int16_t *taps = ip->taps;
    const int out_shift = ip->out_shift, err_shift = ip->err_shift;
    // rs of |G| <= 2^15 is 0 from 17 on
    const int mu_early = ip->mu_shift < 20 ? ip->mu_shift : 20;
    const int mu_late = ip->mu_shift_late < 20 ? ip->mu_shift_late : 20;
    const uint32_t gear = ip->gear_blocks;
    const uint64_t blk0 = ip->block0;
    const int64_t c2 = (int64_t)ip->const_unit * ip->const_unit;
    const bool upd = ip->update_enable != 0;
    const uint32_t nb = (uint32_t)((M + 15) / 16);

    int32_t w[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int32_t val = taps[f * 16 + k];
        if (val < -8192 || val > 8191) flag(err, RANGE_TAP);
        w[k] = clamp32(val, -8192, 8191);
    }
    auto finish = [&]() {
        if (qd == 0) {
#pragma unroll
            for (int k = 0; k < 16; ++k) taps[f * 16 + k] = (int16_t)w[k];
        }
        if (ip->hist_out) {
            uint32_t h = 0u;
            if (lane < 16) {
                const int64_t i = (int64_t)M - 16 + lane;
                if (i >= 0) h = reinterpret_cast<const uint32_t *>(ain)[i];
                else if (hist_in) h = reinterpret_cast<const uint32_t *>(hist_in)[16 + i];
            }
            if (lane < 16) reinterpret_cast<uint32_t *>(ip->hist_out)[lane] = h;
        }
        if (ip->cdc_tail) {
            uint32_t tl = 0u;
            if (lane < 32) {
                const int64_t j = (int64_t)ip->cdc_n - 32 + lane;
                tl = j >= 0 ? reinterpret_cast<const uint32_t *>(ip->cdc_in)[j]
                            : reinterpret_cast<const uint32_t *>(ip->cdc_tail)[32 + j];
            }
            if (lane < 32) reinterpret_cast<uint32_t *>(ip->cdc_tail)[lane] = tl;
        }
    };
    if (nb == 0) {
        finish();
        return;
    }

    // half hh of the digit-d spectrum (N^-1 = -2048 folded in): digit * -2048 =
    // w A + hi B with hi = (w + 64) >> 7; the upper half's first stage is
    // digit * 2^j (its own inputs are the zero padding)
    const int32_t dA = d ? -2048 : 0, dB = d ? 262144 : -2048;
    int32_t W[16];
    auto transform_taps = [&]() {
        sfor<16>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const int32_t hi = (w[k] + 64) >> 7;
            const int32_t v = sext24(w[k]) * dA + sext24(hi) * dB;   // |.| <= 2^17
            W[k] = hh ? tw2_diff<k>(v, 0) : v;
        });
        fwd_stage_n<8, 16>(W);
        fwd_stage_n<4, 16>(W);
        fwd_stage_n<2, 16>(W);
        fwd_stage_n<1, 16>(W);
    };
    transform_taps();
    if (lane < 16) abytes[lane >> 2][68 + (lane & 3)] = 0u;
    uint32_t bad = 0u;
    const int om = (lane >> 1) & 15, opol = lane & 1;   // output / error role (lanes < 32)
    const int32_t dscale = d ? 1 : 128;

    // Symbols 16 b - 16 .. 16 b + 255 of a batch of 16 blocks from b: the lane's
    // p = lane + 64 r (r < 5, p < 272), history before 0 and zeros past M,
    // fetched one batch ahead and waited for at the batch's start.
    uint32_t pre[5];
    const auto ain32 = gptr(reinterpret_cast<const uint32_t *>(ain));
#pragma unroll
    for (int r = 0; r < 5; ++r) {                     // the first batch, with the history
        const int p = lane + 64 * r, i = p - 16;
        uint32_t v = 0u;
        if (p < 272) {
            if (i < 0) {
                if (hist_in) v = gptr(reinterpret_cast<const uint32_t *>(hist_in))[16 + i];
            } else if ((uint64_t)i < M) {
                v = ain32[i];
            }
        }
        pre[r] = v;
    }
    // a later batch (b > 0): every index is at least 0; loads of lanes past M
    // are skipped and their zero applied when the batch is staged
    auto fetch = [&](uint32_t b) {
#pragma unroll
        for (int r = 0; r < 5; ++r) {
            const int p = lane + 64 * r;
            const uint64_t i = 16 * (uint64_t)b - 16 + p;
            if (p < 272 && i < M) pre[r] = ain32[i];
        }
    };

    for (uint32_t b = 0; b < nb; ++b) {
        const int mu_shift = (gear != 0u && blk0 + b >= (uint64_t)gear) ? mu_late : mu_early;   // step schedule
        const int j = (int)(b & 15);
        if (j == 0) {
            // stage the batch's symbols of the four streams as bytes
            wave_lds_sync();
            vmem_wait_all();
#pragma unroll
            for (int r = 0; r < 5; ++r) {
                const int p = lane + 64 * r;
                if (p < 272) {
                    const int64_t i = 16 * (int64_t)b - 16 + p;
                    const uint32_t v = (uint64_t)i < M || i < 0 ? pre[r] : 0u;   // zeros past M
                    if (i >= 0) bad |= v ^ (v << 1);
                    uint8_t *ab = reinterpret_cast<uint8_t *>(&abytes[0][0]);
#pragma unroll
                    for (int c = 0; c < 4; ++c) ab[c * 288 + p] = (uint8_t)(v >> (8 * c));
                }
            }
            fetch(b + 16);                              // the next batch
            wave_lds_sync();
            {   // input spectra of the batch: stream lane % 4, block lane / 4
                const int s1 = lane & 3, jb = lane >> 2;
                const uint4 *src = reinterpret_cast<const uint4 *>(&abytes[s1][4 * jb]);
                int32_t x[32];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const uint4 v4 = src[q];
                    const uint32_t vv[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
                    for (int c = 0; c < 4; ++c)
#pragma unroll
                        for (int e = 0; e < 4; ++e) x[16 * q + 4 * c + e] = sbyte(vv[c], e);
                }
                fnt32_regs<false>(x);
                int4 *dst = reinterpret_cast<int4 *>(&aspec[jb][s1][0]);
#pragma unroll
                for (int q = 0; q < 8; ++q) dst[q] = make_int4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
            }
            wave_lds_sync();
        }
        // products on this half, pair sums over s, inverse stages inside the half
        int32_t Y[16];
        {
            const int4 *A4 = reinterpret_cast<const int4 *>(&aspec[j][S1][16 * hh]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int4 a4 = A4[q];
                Y[4 * q] = mulmod(a4.x, W[4 * q]);
                Y[4 * q + 1] = mulmod(a4.y, W[4 * q + 1]);
                Y[4 * q + 2] = mulmod(a4.z, W[4 * q + 2]);
                Y[4 * q + 3] = mulmod(a4.w, W[4 * q + 3]);
            }
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) Y[k] += xor_lane<8>(Y[k]);   // |.| < 2^17.4
        inv_stage_n<1, 16>(Y);
        inv_stage_n<2, 16>(Y);
        inv_stage_n<4, 16>(Y);
        inv_stage_n<8, 16>(Y);
        // last inverse stage: output 16 + q = y_lo[q] - y_hi[q] 2^-q; half 0 makes
        // outputs q < 8, half 1 outputs q >= 8, each taking the other's value
        int32_t yv[8];
        sfor<8>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const int32_t recv = xor_lane<1>(hh ? Y[i] : Y[8 + i]);
            const int32_t a = hh ? recv : Y[i];
            const int32_t bb = hh ? Y[8 + i] : recv;
            const int32_t t = hh ? neg_inv_tw<8 + i>(bb) : neg_inv_tw<i>(bb);
            int32_t v = sext24(lift_z(a + t)) * dscale;   // |lifted| <= 2^15
            v += xor_lane<2>(v);                           // digits
            v += xor_lane<4>(v);                           // S1 groups
            yv[i] = v;                                     // |.| < 2^23.1
        });
        if ((lane & 14) == 0) {                          // d = 0, S1 = 0: S2 = lane / 16, half hh
            int4 *yd4 = reinterpret_cast<int4 *>(&ybuf[S2][8 * hh]);
            yd4[0] = make_int4(yv[0], yv[1], yv[2], yv[3]);
            yd4[1] = make_int4(yv[4], yv[5], yv[6], yv[7]);
        }
        wave_lds_sync();
        // outputs and RDE errors: lanes < 32, symbol om, streams 2 opol (I), 2 opol + 1 (Q)
        const int64_t m = 16 * (int64_t)b + om;
        const bool valid = lane < 32 && (uint64_t)m < M;
        const int32_t yi = ybuf[2 * opol][om], yq = ybuf[2 * opol + 1][om];
        const int32_t hi_ = clamp32((yi + ((1 << out_shift) >> 1)) >> out_shift, -32768, 32767);
        const int32_t hq_ = clamp32((yq + ((1 << out_shift) >> 1)) >> out_shift, -32768, 32767);
        if (valid)
            gptr(reinterpret_cast<uint32_t *>(outp))[2 * m + opol] = ((uint32_t)hi_ & 0xFFFFu) | ((uint32_t)hq_ << 16);
        if (upd) {
            const int64_t r2 = (int64_t)hi_ * hi_ + (int64_t)hq_ * hq_;
            const int64_t R2 = r2 < 6 * c2 ? 2 * c2 : (r2 < 14 * c2 ? 10 * c2 : 18 * c2);
            int32_t ei = (int32_t)clamp64(rs64((R2 - r2) * hi_, err_shift), -128, 127);
            int32_t eq = (int32_t)clamp64(rs64((R2 - r2) * hq_, err_shift), -128, 127);
            if (!valid) ei = eq = 0;
            if (lane < 32) {
                uint8_t *eb = reinterpret_cast<uint8_t *>(&epsw[0][0]);
                eb[(2 * opol) * 16 + om] = (uint8_t)ei;
                eb[(2 * opol + 1) * 16 + om] = (uint8_t)eq;
            }
            wave_lds_sync();
            // G[k] = sum_m eps_S2[m] a_S1[16 b + m - k] for k = 4 qd + i (i < 4)
            uint32_t e4[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) e4[q] = epsw[S2][q];
            uint32_t dd[6];
            const int q0 = 4 * j + 3 - qd;               // byte 4 q0 = 16 j + 12 - 4 qd
#pragma unroll
            for (int r = 0; r < 6; ++r) dd[r] = abytes[S1][q0 + r];
            int32_t nw[4];
            sfor<4>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int o = 4 - i;                    // a_S1[16 b - k] is byte o of dd
                int32_t gsum = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    gsum = __builtin_amdgcn_sdot4((int)e4[q],
                                                  (int)__builtin_amdgcn_alignbyte(dd[(o >> 2) + q + 1],
                                                                                  dd[(o >> 2) + q], o & 3),
                                                  gsum, false);
                // opaque values: a select of array loads would be folded into one
                // dynamically indexed load, which moves w to scratch memory
                const int32_t c01 = (qd & 1) ? opq(w[4 + i]) : opq(w[i]);
                const int32_t c23 = (qd & 1) ? opq(w[12 + i]) : opq(w[8 + i]);
                const int32_t cur = (qd & 2) ? c23 : c01;
                nw[i] = clamp32(cur + ((gsum + ((1 << mu_shift) >> 1)) >> mu_shift), -8192, 8191);
            });
            sfor<4>([&](auto qc) {                        // every lane of the quad takes all 16 taps
                constexpr int q = decltype(qc)::value;
#pragma unroll
                for (int i = 0; i < 4; ++i) w[4 * q + i] = quad_bcast<q>(nw[i]);
            });
            transform_taps();
        }
        // the next block rewrites the output and error bytes: reads above first
        wave_lds_sync();
        if (b + 1 == nb) finish();
    }
    if ((bad & 0xE0E0E0E0u) != 0u) flag(err, RANGE_SYMBOL);
}

template <int WPG>
__global__ __launch_bounds__(64 * WPG) void aeq_duo_kernel(const AeqItem *items, int nitems,
                                                           AeqItem single, int *err, int prio) {
    aeq_duo_body<WPG>(items, nitems, single, err, prio, blockIdx.x);
}

// One launch for a split plan: its first workgroups run the longest chains in
// form LF at raised priority (they are dispatched first), the others the rest
// of the table in form RF, with WPG waves per workgroup throughout.  Forms:
// 0 (one transform per lane, 2 channels per wave), 3 (two lanes per transform,
// 1 channel per wave), 1 / 2 / 4 (split by polarisation with 1 / 2 / 4 waves per
// half: one workgroup per half, so WPG = 1 / 2 / 4), 5 (split by polarisation,
// one wave per half, both halves in one workgroup: WPG = 2).
__host__ __device__ constexpr unsigned aeq_form_blocks(int form, int n, int wpg) {
    return form == 0 ? (unsigned)((n + 2 * wpg - 1) / (2 * wpg))
         : form == 3 ? (unsigned)((n + wpg - 1) / wpg) : form == 5 ? (unsigned)n : pol_blocks(n);
}
template <int F, int WPG>
__device__ __forceinline__ void aeq_form_body(const AeqItem *items, int n, int *err, int prio, unsigned bid) {
    const AeqItem none{};
    if constexpr (F == 0) aeq_lane_body<WPG>(items, n, none, err, prio, bid);
    else if constexpr (F == 3) aeq_duo_body<WPG>(items, n, none, err, prio, bid);
    else if constexpr (F == 5) {
        static_assert(WPG == 2, "form 5 runs two waves per workgroup");
        aeq_pol_body<4, 2>(items, n, none, err, prio, bid);
    } else aeq_pol_body<4 * WPG>(items, n, none, err, prio, bid);
}
template <int LF, int RF, int WPG>
__global__ __launch_bounds__(64 * WPG) void aeq_split_kernel(const AeqItem *items, int nlong, int nitems,
                                                             int *err, int rest_prio) {
    const unsigned nbl = aeq_form_blocks(LF, nlong, WPG);
    if (blockIdx.x < nbl) aeq_form_body<LF, WPG>(items, nlong, err, 1, blockIdx.x);
    else aeq_form_body<RF, WPG>(items + nlong, nitems - nlong, err, rest_prio, blockIdx.x - nbl);
}

// Direct comparator: y by integer dot products in the time domain, same RDE.
__global__ __launch_bounds__(64) void aeq_direct_kernel(const AeqItem *items, AeqItem single,
                                                        int *err) {
    const AeqItem it = items ? items[blockIdx.x] : single;
    const int lane = threadIdx.x;
    const int pos = lane & 31;
    const int s1 = lane >> 4, kk = lane & 15;
    __shared__ int16_t tapl[256];
    __shared__ uint32_t epsw[16];
    __shared__ uint32_t winw[36];

    int32_t w[4];
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
        int32_t v = it.taps[(s1 * 4 + s2) * 16 + kk];
        if (v < -8192 || v > 8191) flag(err, RANGE_TAP);
        w[s2] = clamp32(v, -8192, 8191);
    }
    const uint64_t M = it.m;
    if (M == 0) {
        aeq_finish(it, lane, w, err);
        return;
    }
    if (lane < 4) winw[32 + lane] = 0u;
    const int64_t nblocks = (int64_t)((M + 15) / 16);
    const int c2 = it.const_unit * it.const_unit;
    uint32_t win = aeq_load(it, -16 + pos, err);
    // output ownership: lane = (S2 = lane >> 4, j = lane & 15)
    const int o2 = lane >> 4, oj = lane & 15;

    for (int64_t b = 0; b < nblocks; ++b) {
        uint32_t nxt = pos >= 16 ? aeq_load(it, 16 * b + pos, err) : 0u;
        if (lane < 32) {
            uint8_t *wb = reinterpret_cast<uint8_t *>(winw);
#pragma unroll
            for (int c = 0; c < 4; ++c) wb[c * 32 + pos] = (uint8_t)(win >> (8 * c));
        }
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) tapl[(s1 * 4 + s2) * 16 + kk] = (int16_t)w[s2];
        __syncthreads();
        // y_S2[16b + j] = sum_S1 sum_k w[S1][S2][k] * a_S1[16 b + j - k]
        int32_t y = 0;
#pragma unroll
        for (int a1 = 0; a1 < 4; ++a1) {
            const uint8_t *wb = reinterpret_cast<const uint8_t *>(winw) + a1 * 32 + 16 + oj;
#pragma unroll
            for (int k = 0; k < 16; ++k) y += (int32_t)tapl[(a1 * 4 + o2) * 16 + k] * (int8_t)wb[-k];
        }
        int32_t yh = (int32_t)clamp64(rs64((int64_t)y, it.out_shift), -32768, 32767);
        // gather the 4 streams of symbol j into lanes j (+16, +32, +48 hold S2 = 1..3)
        int32_t ys[4];
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) ys[s2] = __shfl(yh, s2 * 16 + oj);
        const int64_t m = 16 * b + oj;
        const bool valid = (uint64_t)m < M;
        if (valid && lane < 16) {
            uint2 o;
            o.x = ((uint32_t)ys[0] & 0xFFFFu) | ((uint32_t)ys[1] << 16);
            o.y = ((uint32_t)ys[2] & 0xFFFFu) | ((uint32_t)ys[3] << 16);
            gptr(reinterpret_cast<uint64_t *>(it.out))[m] = (uint64_t)o.x | ((uint64_t)o.y << 32);
        }
        if (it.update_enable) {
            uint32_t epack = 0;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                int64_t yi = ys[2 * p], yq = ys[2 * p + 1];
                int64_t r2 = yi * yi + yq * yq;
                int64_t R2 = r2 < 6LL * c2 ? 2LL * c2 : (r2 < 14LL * c2 ? 10LL * c2 : 18LL * c2);
                int64_t e = R2 - r2;
                int32_t ei = (int32_t)clamp64(rs64(e * yi, it.err_shift), -128, 127);
                int32_t eq = (int32_t)clamp64(rs64(e * yq, it.err_shift), -128, 127);
                epack |= ((uint32_t)ei & 0xFFu) << (16 * p);
                epack |= ((uint32_t)eq & 0xFFu) << (16 * p + 8);
            }
            if (!valid) epack = 0u;
            if (lane < 16) {
                uint8_t *eb = reinterpret_cast<uint8_t *>(epsw);
#pragma unroll
                for (int c = 0; c < 4; ++c) eb[c * 16 + oj] = (uint8_t)(epack >> (8 * c));
            }
            __syncthreads();
            const int off = s1 * 32 + 16 - kk;
            uint32_t d[5];
#pragma unroll
            for (int r = 0; r < 5; ++r) d[r] = winw[(off >> 2) + r];
            uint32_t xs[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) xs[q] = __builtin_amdgcn_alignbyte(d[q + 1], d[q], off & 3);
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) {
                int32_t g = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    g = __builtin_amdgcn_sdot4((int)epsw[s2 * 4 + q], (int)xs[q], g, false);
                w[s2] = clamp32(w[s2] + (int32_t)rs64((int64_t)g, step_shift(it, it.block0 + (uint64_t)b)), -8192, 8191);
            }
        }
        __syncthreads();
        uint32_t slid = (uint32_t)__shfl((int)win, (lane & 32) | ((pos + 16) & 31));
        win = pos < 16 ? slid : nxt;
    }
    aeq_finish(it, lane, w, err);
}

}  // namespace

namespace fnti {

static_assert(RANGE_STALL == kFlagStall, "stall flag bit");

// Producer waves of the fused kernel per AEQ form: as many as waves per
// polarisation half, one per SIMD the consumers run on.
template <int LPT>
static hipError_t fused_kernel_caps(int *per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, cdc_aeq_fused_kernel<LPT, LPT / 4, 2>,
                                                        64 * (3 * (LPT / 4)), 0);
}

int fused_capacity(int lpt) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e = lpt == 4 ? fused_kernel_caps<4>(&per) : lpt == 8 ? fused_kernel_caps<8>(&per)
                 : lpt == 16 ? fused_kernel_caps<16>(&per) : hipErrorInvalidValue;
    return e == hipSuccess ? per * cus : 0;
}

unsigned fused_split_grid(int n) { return pol_blocks(n); }

hipError_t launch_fused(const CdcItem *citems, const AeqItem *aitems, int n, const CdcItem &cs,
                        const AeqItem &as, int lpt, uint32_t *queue, unsigned grid, int nprio, int *err,
                        hipStream_t s, bool split_halves, uint32_t spin_limit) {
    const int total = citems ? n : 1;
    if (total <= 0) return hipSuccess;
    if ((citems == nullptr) != (aitems == nullptr) || n > (1 << 26) || grid == 0) return hipErrorInvalidValue;
    if (split_halves) {
        // one workgroup per half: the pairs of every run of 16 workgroups
        if (queue || grid != pol_blocks(total)) return hipErrorInvalidValue;
        switch (lpt) {
        case 4: cdc_aeq_fused_kernel<4, 1, 1><<<grid, 128, 0, s>>>(citems, aitems, n, cs, as, nullptr, nprio, err, spin_limit); break;
        case 8: cdc_aeq_fused_kernel<8, 2, 1><<<grid, 256, 0, s>>>(citems, aitems, n, cs, as, nullptr, nprio, err, spin_limit); break;
        case 16: cdc_aeq_fused_kernel<16, 4, 1><<<grid, 512, 0, s>>>(citems, aitems, n, cs, as, nullptr, nprio, err, spin_limit); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (queue ? grid > (unsigned)total : grid != (unsigned)total) return hipErrorInvalidValue;
    switch (lpt) {
    case 4: cdc_aeq_fused_kernel<4, 1, 2><<<grid, 192, 0, s>>>(citems, aitems, n, cs, as, queue, nprio, err, spin_limit); break;
    case 8: cdc_aeq_fused_kernel<8, 2, 2><<<grid, 384, 0, s>>>(citems, aitems, n, cs, as, queue, nprio, err, spin_limit); break;
    case 16: cdc_aeq_fused_kernel<16, 4, 2><<<grid, 768, 0, s>>>(citems, aitems, n, cs, as, queue, nprio, err, spin_limit); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_transform(const uint32_t *x, uint32_t *X, size_t batch, int t, int log2n,
                            int alpha_kind, bool inverse, int *err, hipStream_t s) {
    const uint64_t total = (uint64_t)batch << log2n;
    if (total == 0) return hipSuccess;
    const unsigned threads = 256;
    // enough workgroups to fill 256 CUs many times over; each thread then
    // loops over the batch (see fnt_transform_kernel)
    const unsigned grid = (unsigned)std::min<uint64_t>((total + threads - 1) / threads, 8192);
#define FNT_LAUNCH(Q, L, S)                                                                   \
    do {                                                                                      \
        if (inverse)                                                                          \
            fnt_transform_kernel<Q, L, S, true><<<grid, threads, 0, s>>>(x, X, total, err);  \
        else                                                                                  \
            fnt_transform_kernel<Q, L, S, false><<<grid, threads, 0, s>>>(x, X, total, err); \
    } while (0)
    // N = order of the radix: 2^(t+1) for alpha = 2, 2^(t+2) for alpha = sqrt 2
    if (t == 2 && log2n == 3 && alpha_kind == FNT_ALPHA_2) FNT_LAUNCH(4, 3, false);
    else if (t == 2 && log2n == 4 && alpha_kind == FNT_ALPHA_SQRT2) FNT_LAUNCH(4, 4, true);
    else if (t == 3 && log2n == 4 && alpha_kind == FNT_ALPHA_2) FNT_LAUNCH(8, 4, false);
    else if (t == 3 && log2n == 5 && alpha_kind == FNT_ALPHA_SQRT2) FNT_LAUNCH(8, 5, true);
    else if (t == 4 && log2n == 5 && alpha_kind == FNT_ALPHA_2) FNT_LAUNCH(16, 5, false);
    else if (t == 4 && log2n == 6 && alpha_kind == FNT_ALPHA_SQRT2) FNT_LAUNCH(16, 6, true);
    else return hipErrorInvalidValue;
#undef FNT_LAUNCH
    return hipGetLastError();
}

hipError_t launch_cdc(const CdcItem *items, int nitems, const CdcItem &single,
                      uint64_t total_blocks, uint64_t total_chunks, int variant,
                      int waves_per_group, int blocks_per_wave, bool with_z, int *err,
                      hipStream_t s) {
    if (total_blocks == 0) return hipSuccess;
    if (waves_per_group < 1 || waves_per_group > 4) return hipErrorInvalidValue;
    if (variant == 0 && !with_z) {
        if (total_chunks == 0) return hipErrorInvalidValue;
        const uint64_t grid = (total_chunks + waves_per_group - 1) / waves_per_group;
        if (grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
        switch (waves_per_group) {
        case 1: cdc_lane_kernel<1><<<(unsigned)grid, 64, 0, s>>>(items, nitems, single, total_chunks, err); break;
        case 2: cdc_lane_kernel<2><<<(unsigned)grid, 128, 0, s>>>(items, nitems, single, total_chunks, err); break;
        case 3: cdc_lane_kernel<3><<<(unsigned)grid, 192, 0, s>>>(items, nitems, single, total_chunks, err); break;
        default: cdc_lane_kernel<4><<<(unsigned)grid, 256, 0, s>>>(items, nitems, single, total_chunks, err); break;
        }
        return hipGetLastError();
    }
    if (variant == 2 && !with_z) {
        if (total_chunks == 0) return hipErrorInvalidValue;
        const uint64_t grid = (total_chunks + waves_per_group - 1) / waves_per_group;
        if (grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
        switch (waves_per_group) {
        case 1: cdc_direct_kernel<1><<<(unsigned)grid, 64, 0, s>>>(items, nitems, single, total_chunks, err); break;
        case 2: cdc_direct_kernel<2><<<(unsigned)grid, 128, 0, s>>>(items, nitems, single, total_chunks, err); break;
        case 3: cdc_direct_kernel<3><<<(unsigned)grid, 192, 0, s>>>(items, nitems, single, total_chunks, err); break;
        default: cdc_direct_kernel<4><<<(unsigned)grid, 256, 0, s>>>(items, nitems, single, total_chunks, err); break;
        }
        return hipGetLastError();
    }
    if (variant != 0 && variant != 1) return hipErrorInvalidValue;
    if (blocks_per_wave < 1) return hipErrorInvalidValue;
    const uint64_t waves = (total_blocks + blocks_per_wave - 1) / blocks_per_wave;
    const uint64_t grid = (waves + waves_per_group - 1) / waves_per_group;
    if (grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
    const unsigned threads = 64u * (unsigned)waves_per_group;
    if (with_z)
        cdc_kernel<true><<<(unsigned)grid, threads, 0, s>>>(items, nitems, single, total_blocks,
                                                            blocks_per_wave, err);
    else
        cdc_kernel<false><<<(unsigned)grid, threads, 0, s>>>(items, nitems, single, total_blocks,
                                                             blocks_per_wave, err);
    return hipGetLastError();
}

static int split_wpg(int form_long) { return (form_long == 2 || form_long == 5) ? 2 : form_long == 4 ? 4 : 1; }

hipError_t launch_aeq_split(const AeqItem *items, int nlong, int nitems, int form_long, int form_rest,
                           int *err, hipStream_t s, bool rest_high_priority) {
    if (!items || nlong <= 0 || nlong >= nitems || nitems > (1 << 26)) return hipErrorInvalidValue;
    const int wpg = split_wpg(form_long);
    const unsigned grid = aeq_form_blocks(form_long, nlong, wpg) + aeq_form_blocks(form_rest, nitems - nlong, wpg);
#define FNT_SPLIT(L, R, W)                                                                     \
    if (form_long == L && form_rest == R) {                                                    \
        aeq_split_kernel<L, R, W><<<grid, 64 * W, 0, s>>>(items, nlong, nitems, err, rest_high_priority ? 1 : 0);           \
        return hipGetLastError();                                                              \
    }
    FNT_SPLIT(1, 0, 1) FNT_SPLIT(1, 3, 1) FNT_SPLIT(3, 0, 1)
    FNT_SPLIT(2, 0, 2) FNT_SPLIT(2, 3, 2) FNT_SPLIT(4, 0, 4) FNT_SPLIT(4, 3, 4)
    FNT_SPLIT(5, 0, 2) FNT_SPLIT(5, 3, 2) FNT_SPLIT(2, 5, 2)
#undef FNT_SPLIT
    return hipErrorInvalidValue;
}

bool aeq_split_fusable(int form_long, int form_rest) {
    return ((form_long == 1 || form_long == 2 || form_long == 4 || form_long == 5) &&
            (form_rest == 0 || form_rest == 3)) ||
           (form_long == 3 && form_rest == 0) || (form_long == 2 && form_rest == 5);
}

hipError_t launch_aeq(const AeqItem *items, int nitems, const AeqItem &single, int variant,
                      int waves_per_pol, int *err, hipStream_t s, bool high_priority) {
    const int prio = high_priority ? 1 : 0;
    const int n = items ? nitems : 1;
    if (n <= 0) return hipSuccess;
    if (n > (1 << 26)) return hipErrorInvalidValue;    // grid sizes stay far below 2^31
    if (variant == 0) {
        if (waves_per_pol == 0)
            aeq_lane_kernel<1><<<(n + 1) / 2, 64, 0, s>>>(items, n, single, err, prio);
        else if (waves_per_pol == 3)
            aeq_duo_kernel<1><<<n, 64, 0, s>>>(items, n, single, err, prio);
        else if (waves_per_pol == 1)
            aeq_pol_kernel<4><<<pol_blocks(n), 64, 0, s>>>(items, n, single, err, prio);
        else if (waves_per_pol == 2)
            aeq_pol_kernel<8><<<pol_blocks(n), 128, 0, s>>>(items, n, single, err, prio);
        else if (waves_per_pol == 4)
            aeq_pol_kernel<16><<<pol_blocks(n), 256, 0, s>>>(items, n, single, err, prio);
        else if (waves_per_pol == 5)
            aeq_pol_kernel<4, 2><<<n, 128, 0, s>>>(items, n, single, err, prio);
        else
            return hipErrorInvalidValue;
    } else if (variant == 1) {
        aeq_direct_kernel<<<n, 64, 0, s>>>(items, single, err);
    } else if (variant == 2) {
        aeq_fnt_kernel<false><<<n, 64, 0, s>>>(items, single, err);
    } else if (variant == 3) {
        aeq_fnt_kernel<true><<<n, 64, 0, s>>>(items, single, err);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fnti

#if FNT_COUNT_PRODUCTS
// Counting build only: read (and with reset, clear) the product counters.
extern "C" int fnt_debug_product_counts(uint64_t *cdc, uint64_t *aeq, int reset) {
    unsigned long long h[2] = {0, 0};
    if (hipDeviceSynchronize() != hipSuccess) return FNT_E_DEVICE;
    if (hipMemcpyFromSymbol(h, HIP_SYMBOL(g_fnt_products), sizeof h) != hipSuccess) return FNT_E_DEVICE;
    if (cdc) *cdc = h[0];
    if (aeq) *aeq = h[1];
    if (reset) {
        const unsigned long long z[2] = {0, 0};
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_fnt_products), z, sizeof z) != hipSuccess) return FNT_E_DEVICE;
    }
    return FNT_OK;
}
#endif
