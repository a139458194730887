// fnt_cdc_long: FNT-CDC with a 128-point transform for up to 65 taps.
//
// The paper's CDC block is N = 64 with 32 new instants, so overlap-save holds
// at most 33 taps.  Fibres longer than about 40 km at 40 GBaud want more.  This
// variant takes N = 128 (64 new instants per block) with a radix of order 128
// modulo F = 65537, alpha = 4938, a square root of the CDC's sqrt 2 (4080).
//
// A 65-tap convolution of 5-bit samples with 6-bit taps reaches
// 65 * 1008 = 65520 per component, beyond the Eq. (5) bound (F - 1) / 2.  The
// taps are therefore split into two balanced 3-bit digits, h = 8 hi + lo with
// lo in [-4, 3] and hi in [-4, 4]; each digit's convolution stays within
// 65 * (4 * 16 + 4 * 16) = 8320.  Each goes through the complex packing of
// Eqs. (7)-(8) (u = x_r + 2^8 x_i, v = x_r - 2^8 x_i, products with the digit's
// two tap spectra, inverse of P + Q and of P - Q); the centred results are
// combined as z = 8 z_hi + z_lo, the exact complex convolution.
//
// With N = 128 the constants of Eqs. (7)-(8) times N^-1 = -2^9 become
// z = -256 IFNT'(P + Q) and z^ = -IFNT'(P - Q) (IFNT' unnormalised).
//
// One wave per block: lane l holds window positions l and l + 64 (instants
// 64 b - 64 + l and 64 b + l); the transform stages at distance 64 stay in the
// lane, the others exchange lanes l ^ h.  Each wave runs kBlocksPerWave
// consecutive blocks after computing the four tap-digit spectra once.
#include <hip/hip_runtime.h>

#include "fnt_common.hpp"
#include "fnt_device.hpp"

using namespace fntd;
using namespace fnti;

namespace {

constexpr int kBlocksPerWave = 16;
constexpr int kWavesPerGroup = 4;
constexpr uint32_t kF = 65537u;
constexpr uint32_t kAlpha128 = 4938u;

struct Pow128 {
    int32_t f[128];   // alpha^e
    int32_t i[128];   // alpha^-e
};
constexpr Pow128 make_pow128() {
    Pow128 t{};
    uint64_t a = 1, b = 1;
    uint64_t inv = 1;                                    // alpha^-1 = alpha^127
    for (int e = 0; e < 127; ++e) inv = inv * kAlpha128 % kF;
    for (int e = 0; e < 128; ++e) {
        t.f[e] = (int32_t)a;
        t.i[e] = (int32_t)b;
        a = a * kAlpha128 % kF;
        b = b * inv % kF;
    }
    return t;
}
__constant__ Pow128 kPow128 = make_pow128();

struct LongParams {
    int8_t taps[FNT_MAX_CDC_LONG_TAPS][2];
    int32_t ntaps;
    int32_t shift;
    int32_t phase;
};

__device__ __forceinline__ void flag_long(int *err, int bit) {
    if (err) atomicOr(err, bit);
}

// Lane exchange at distance H (1 .. 32) inside the wave.
template <int H>
__device__ __forceinline__ int32_t xl(int32_t v) {
    if constexpr (H == 32) return __shfl_xor(v, 32);
    else return xor_lane<H>(v);
}

// Per-lane twiddles: forward stage h (h = 64 in the lane, then 32 .. 1) uses
// alpha^((64 / h) (l mod h)); the inverse uses the reciprocal powers.
struct Twiddles {
    int32_t f[7];
    int32_t i[7];
};
__device__ __forceinline__ Twiddles lane_twiddles(int l) {
    Twiddles t;
#pragma unroll
    for (int s = 0; s < 7; ++s) {
        const int h = 64 >> s;
        const int e = (64 / h) * (l & (h - 1));
        t.f[s] = kPow128.f[e];
        t.i[s] = kPow128.i[e];
    }
    return t;
}

// One forward cross-lane DIF stage at distance H: lower lane a + p, upper lane
// (p - a) c.  Inputs |.| < 2^22; the upper output < 2^16 + 2^14.
template <int H>
__device__ __forceinline__ int32_t fwd_stage(int32_t a, int32_t c, bool up) {
    const int32_t p = xl<H>(a);
    return up ? mulmod(p - a, c) : a + p;
}

// DIF FNT128: natural positions (l, l + 64) in x[0], x[1] -> bins in the order
// the inverse expects.  |in| <= 2^13: out |.| < 2^22.3.
__device__ __forceinline__ void fwd128(int32_t (&x)[2], int l, const Twiddles &tw) {
    const int32_t a = x[0], b = x[1];
    x[0] = a + b;
    x[1] = mulmod(a - b, tw.f[0]);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        x[r] = fwd_stage<32>(x[r], tw.f[1], (l & 32) != 0);
        x[r] = fwd_stage<16>(x[r], tw.f[2], (l & 16) != 0);
        x[r] = fwd_stage<8>(x[r], tw.f[3], (l & 8) != 0);
        x[r] = fwd_stage<4>(x[r], tw.f[4], (l & 4) != 0);
        x[r] = fwd_stage<2>(x[r], tw.f[5], (l & 2) != 0);
        x[r] = fwd_stage<1>(x[r], tw.f[6], (l & 1) != 0);
    }
}

// One inverse DIT stage at distance H: t = (upper input) c; lower lane a + t,
// upper lane p - t.
template <int H>
__device__ __forceinline__ int32_t inv_stage(int32_t a, int32_t c, bool up) {
    const int32_t p = xl<H>(a);
    const int32_t t = mulmod(up ? a : p, c);
    return up ? p - t : a + t;
}

// DIT inverse (unnormalised, alpha^-1) from the forward order back to natural
// positions, keeping position l + 64 only.  |in| < 2^18: out |.| < 2^20.
__device__ __forceinline__ int32_t inv128_upper(int32_t (&x)[2], int l, const Twiddles &tw) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        x[r] = inv_stage<1>(x[r], tw.i[6], (l & 1) != 0);
        x[r] = inv_stage<2>(x[r], tw.i[5], (l & 2) != 0);
        x[r] = inv_stage<4>(x[r], tw.i[4], (l & 4) != 0);
        x[r] = inv_stage<8>(x[r], tw.i[3], (l & 8) != 0);
        x[r] = inv_stage<16>(x[r], tw.i[2], (l & 16) != 0);
        x[r] = inv_stage<32>(x[r], tw.i[1], (l & 32) != 0);
    }
    return x[0] - mulmod(x[1], tw.i[0]);
}

__device__ __forceinline__ int32_t digit_lo(int32_t h) { return ((h + 4) & 7) - 4; }
__device__ __forceinline__ int32_t digit_hi(int32_t h) { return (h - digit_lo(h)) >> 3; }

__device__ __forceinline__ int32_t sat5_rs(int32_t z, int s) {
    const int32_t r = (int32_t)(((int64_t)z + ((int64_t)1 << s >> 1)) >> s);
    return r < -16 ? -16 : (r > 15 ? 15 : r);
}

__device__ __forceinline__ uint32_t load_instant(const int8_t *in, uint64_t n, int64_t i) {
    return (i >= 0 && (uint64_t)i < n) ? reinterpret_cast<const uint32_t *>(in)[i] : 0u;
}

__global__ __launch_bounds__(64 * kWavesPerGroup) void cdc_long_kernel(const int8_t *__restrict__ in, uint64_t n,
                                                                      LongParams prm, int32_t *z_out,
                                                                      int8_t *a_out, uint64_t nblocks,
                                                                      int *err) {
    const int l = threadIdx.x & 63;
    const uint64_t wave = (uint64_t)blockIdx.x * kWavesPerGroup + (threadIdx.x >> 6);
    const uint64_t b0 = wave * kBlocksPerWave;
    if (b0 >= nblocks) return;
    const Twiddles tw = lane_twiddles(l);

    // tap-digit spectra: Hp[d] = FNT(h_r,d + 2^8 h_i,d), Hm[d] = FNT(h_r,d - 2^8 h_i,d)
    int32_t Hp[2][2], Hm[2][2];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int k = l + 64 * r;
            int32_t hr = 0, hi = 0;
            if (k < prm.ntaps) {
                hr = prm.taps[k][0];
                hi = prm.taps[k][1];
            }
            const int32_t dr = d ? digit_lo(hr) : digit_hi(hr);
            const int32_t di = d ? digit_lo(hi) : digit_hi(hi);
            Hp[d][r] = dr + 256 * di;                    // |.| <= 1028
            Hm[d][r] = dr - 256 * di;
        }
        fwd128(Hp[d], l, tw);
        fwd128(Hm[d], l, tw);
    }

    bool bad = false;
    const uint64_t b1 = b0 + kBlocksPerWave < nblocks ? b0 + kBlocksPerWave : nblocks;
    for (uint64_t b = b0; b < b1; ++b) {
        const int64_t i_new = (int64_t)(64 * b) + l;    // instant at window position l + 64
        const uint32_t w0 = load_instant(in, n, i_new - 64), w1 = load_instant(in, n, i_new);
        bad |= ((w0 ^ (w0 << 1)) & 0xE0E0E0E0u) != 0u || ((w1 ^ (w1 << 1)) & 0xE0E0E0E0u) != 0u;
        int32_t z[4];
        uint32_t a_word = 0;
#pragma unroll
        for (int pol = 0; pol < 2; ++pol) {
            const int32_t xr0 = (int8_t)(w0 >> (16 * pol)), xi0 = (int8_t)(w0 >> (16 * pol + 8));
            const int32_t xr1 = (int8_t)(w1 >> (16 * pol)), xi1 = (int8_t)(w1 >> (16 * pol + 8));
            int32_t U[2] = {xr0 + 256 * xi0, xr1 + 256 * xi1};   // Eq. (7) packing, |.| <= 4112
            int32_t V[2] = {xr0 - 256 * xi0, xr1 - 256 * xi1};   // Eq. (8) packing
            fwd128(U, l, tw);
            fwd128(V, l, tw);
            int32_t zr = 0, zi = 0;
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                int32_t S[2], D[2];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int32_t P = mulmod(U[r], Hp[d][r]);     // |.| < 2^16 + 2^14
                    const int32_t Q = mulmod(V[r], Hm[d][r]);
                    S[r] = P + Q;
                    D[r] = P - Q;
                }
                const int32_t s = inv128_upper(S, l, tw);
                const int32_t t = inv128_upper(D, l, tw);
                // Eq. (7): z = -256 IFNT'(P + Q); Eq. (8): z^ = -IFNT'(P - Q); |digit z| <= 8320
                const int32_t dr = lift_loose(mulmod(s, -256));
                const int32_t di = lift_loose(-t);
                zr = d ? zr + dr : 8 * dr;
                zi = d ? zi + di : 8 * di;
            }
            z[2 * pol] = zr;
            z[2 * pol + 1] = zi;
            a_word |= ((uint32_t)sat5_rs(zr, prm.shift) & 0xFFu) << (16 * pol);
            a_word |= ((uint32_t)sat5_rs(zi, prm.shift) & 0xFFu) << (16 * pol + 8);
        }
        if ((uint64_t)i_new < n) {
            if (z_out)
                reinterpret_cast<int4 *>(z_out)[i_new] = make_int4(z[0], z[1], z[2], z[3]);
            if (a_out && i_new >= prm.phase && ((i_new - prm.phase) & 1) == 0)
                reinterpret_cast<uint32_t *>(a_out)[(i_new - prm.phase) >> 1] = a_word;
        }
    }
    if (bad) flag_long(err, RANGE_SAMPLE);
}

}  // namespace

extern "C" int fnt_cdc_long(const int8_t *in, uint64_t n, const int8_t *host_taps, int ntaps, int requant_shift,
                            int decim_phase, int32_t *out_exact, int8_t *out_1sps, void *stream) {
    if (ntaps < 1 || ntaps > FNT_MAX_CDC_LONG_TAPS)
        return fail(FNT_E_INVAL, "fnt_cdc_long: %d taps (1 .. %d)", ntaps, FNT_MAX_CDC_LONG_TAPS);
    if (!host_taps) return fail(FNT_E_INVAL, "fnt_cdc_long: NULL taps");
    if (requant_shift < 0 || requant_shift > 16) return fail(FNT_E_INVAL, "fnt_cdc_long: shift %d", requant_shift);
    if (decim_phase != 0 && decim_phase != 1) return fail(FNT_E_INVAL, "fnt_cdc_long: phase %d", decim_phase);
    LongParams prm{};
    for (int k = 0; k < ntaps; ++k) {
        const int8_t hr = host_taps[2 * k], hi = host_taps[2 * k + 1];
        if (hr < -32 || hr > 31 || hi < -32 || hi > 31)
            return fail(FNT_E_RANGE, "fnt_cdc_long: tap %d = (%d, %d) outside 6 bit", k, hr, hi);
        prm.taps[k][0] = hr;
        prm.taps[k][1] = hi;
    }
    prm.ntaps = ntaps;
    prm.shift = requant_shift;
    prm.phase = decim_phase;
    if (n == 0) return FNT_OK;
    if (!in) return fail(FNT_E_INVAL, "fnt_cdc_long: NULL input");
    if (!aligned(in, 4) || (out_exact && !aligned(out_exact, 16)) || (out_1sps && !aligned(out_1sps, 4)))
        return fail(FNT_E_INVAL, "fnt_cdc_long: misaligned buffer");
    int *err = nullptr;
    int rc = device_err_flag(&err);
    if (rc) return rc;
    const uint64_t nblocks = (n + 63) / 64;
    const uint64_t waves = (nblocks + kBlocksPerWave - 1) / kBlocksPerWave;
    const uint64_t grid = (waves + kWavesPerGroup - 1) / kWavesPerGroup;
    if (grid > 0x7FFFFFFFull) return fail(FNT_E_INVAL, "fnt_cdc_long: %llu instants", (unsigned long long)n);
    cdc_long_kernel<<<(unsigned)grid, 64 * kWavesPerGroup, 0, (hipStream_t)stream>>>(in, n, prm, out_exact,
                                                                                      out_1sps, nblocks, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "fnt_cdc_long launch");
    return FNT_OK;
}
