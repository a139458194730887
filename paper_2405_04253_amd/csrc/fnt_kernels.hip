// gfx950 kernels of the FNT-CDC + FNT-AEQ receiver path.
//
//  * fnt_transform_kernel : batched Eq. (1) / Eq. (2) transforms (Fig. 1 case,
//    the AEQ's N = 32 / alpha = 2 and the CDC's N = 64 / alpha = sqrt 2).
//  * cdc_kernel           : overlap-save FNT-CDC (Fig. 2), complex product through
//    the two real Fermat-domain products of Eqs. (7)-(8), exact centred lift,
//    resampling to 1 sample/symbol and requantisation to 5 bit.
//  * aeq_fnt_kernel       : FNT-AEQ (Fig. 3): 4x4 real MIMO filtering in the
//    Fermat domain with 14-bit taps split into two 7-bit digit groups, the RDE
//    error of Eq. (6) and the block tap update; one wave64 per channel.
//  * aeq_direct_kernel    : the same AEQ with time-domain integer dot products,
//    a comparator with bit-identical output.
#include <hip/hip_runtime.h>

#include "fnt_device.hpp"
#include "fnt_internal.hpp"

using namespace fntd;
using fnti::AeqItem;
using fnti::CdcItem;

namespace {

__device__ __forceinline__ void flag(int *err, int bit) {
    if (err) atomicOr(err, bit);
}

// ---------------------------------------------------------------- transforms --

constexpr uint32_t pow_mod(uint32_t b, uint32_t e, uint32_t m) {
    uint64_t r = 1, x = b % m;
    while (e) {
        if (e & 1) r = r * x % m;
        x = x * x % m;
        e >>= 1;
    }
    return (uint32_t)r;
}

template <int Q, int LOGN, bool SQRT2, bool INV>
__global__ __launch_bounds__(256) void fnt_transform_kernel(const uint32_t *x, uint32_t *X,
                                                            uint64_t total, int *err) {
    using FF = Field<Q>;
    constexpr int N = 1 << LOGN;
    constexpr uint32_t NINV = pow_mod(N, FF::F - 2, FF::F);
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int pos = lane & (N - 1);
    const bool valid = gid < total;
    const uint64_t base = gid - (uint64_t)pos;
    uint32_t v = 0;
    if (valid) {
        v = x[INV ? base + (uint64_t)bitrev(pos, LOGN) : gid];
        if (v >= FF::F) {
            flag(err, RANGE_RESIDUE);
            v %= FF::F;
        }
    }
    uint64_t dst;
    if constexpr (!INV) {
        v = fwd_xlane<Q, LOGN, SQRT2>(v, lane);
        dst = base + (uint64_t)bitrev(pos, LOGN);
    } else {
        v = FF::mul(inv_xlane<Q, LOGN, SQRT2>(v, lane), NINV);
        dst = gid;
    }
    if (valid) X[dst] = v;
}

// ----------------------------------------------------------------------- CDC --

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

// Tap spectra H+ = FNT64(h_r + 256 h_i), H- = FNT64(h_r - 256 h_i) in lane order
// (lane l holds bin bitrev(l)), the per-channel factors of Eqs. (7)-(8).
// `taps` points at the item's int8[32][2] taps (device table or kernel argument).
__device__ __forceinline__ void cdc_spectra(const int8_t *taps, int ntaps, int lane, uint32_t &hp,
                                            uint32_t &hm) {
    using FF = Field<16>;
    int hr = 0, hi = 0;
    if (lane < ntaps) {
        hr = taps[2 * lane];
        hi = taps[2 * lane + 1];
    }
    hp = fwd_xlane<16, 6, true>(FF::from_int(hr + 256 * hi), lane);
    hm = fwd_xlane<16, 6, true>(FF::from_int(hr - 256 * hi), lane);
}

template <bool WITH_Z>
__global__ __launch_bounds__(256) void cdc_kernel(const CdcItem *items, int nitems,
                                                  CdcItem single, uint64_t total_blocks,
                                                  int blocks_per_wave, int *err) {
    using FF = Field<16>;
    const int lane = threadIdx.x & 63;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t b_begin = wave * (uint64_t)blocks_per_wave;
    if (b_begin >= total_blocks) return;
    uint64_t b_end = b_begin + (uint64_t)blocks_per_wave;
    if (b_end > total_blocks) b_end = total_blocks;

    // item holding global block b_begin: the last one with block0 <= b_begin
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
    uint32_t hp, hm;
    cdc_spectra(items ? &items[idx].taps[0][0] : &single.taps[0][0], it.ntaps, lane, hp, hm);
    bool have_prev = false;
    uint32_t prev = 0;

    for (uint64_t b = b_begin; b < b_end; ++b) {
        while (b >= it_end) {  // next item (skips items with n == 0)
            ++idx;
            it = items[idx];
            it_end = it.block0 + fnti::cdc_blocks(it.n);
            have_prev = false;
            cdc_spectra(&items[idx].taps[0][0], it.ntaps, lane, hp, hm);
        }
        const int64_t lb = (int64_t)(b - it.block0);
        // window: instants [32 lb - 32, 32 lb + 32); lanes 0..31 reuse the
        // previous block's new half when this wave just processed it
        const int64_t inst = 32 * lb - 32 + lane;
        uint32_t carried = (uint32_t)__shfl((int)prev, (lane + 32) & 63);
        uint32_t w = (have_prev && lane < 32) ? carried : cdc_load(it, inst);
        if (!bytes_5bit(w)) flag(err, RANGE_SAMPLE);
        prev = w;
        have_prev = true;

        uint32_t u[2], v[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            int xr = sbyte(w, 2 * p), xi = sbyte(w, 2 * p + 1);
            u[p] = fwd_xlane<16, 6, true>(FF::from_int(xr + 256 * xi), lane);
            v[p] = fwd_xlane<16, 6, true>(FF::from_int(xr - 256 * xi), lane);
        }
        int32_t z[4];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            uint32_t P = FF::mul(u[p], hp), Qv = FF::mul(v[p], hm);
            uint32_t S = inv_xlane<16, 6, true>(FF::add(P, Qv), lane);
            uint32_t D = inv_xlane<16, 6, true>(FF::sub(P, Qv), lane);
            // Eq. (7): z = -2^15 * 64^-1 * S' = -512 S'; Eq. (8): z^ = -2^7 * 64^-1 * D' = -2 D'
            z[2 * p] = FF::lift(FF::neg(FF::mulpow2(S, 9)));
            z[2 * p + 1] = FF::lift(FF::neg(FF::mulpow2(D, 1)));
        }
        if (lane >= 32) {
            const int64_t i = 32 * lb + (lane - 32);
            if ((uint64_t)i < it.n) {
                if (WITH_Z && it.z_out) {
                    int4 zz = make_int4(z[0], z[1], z[2], z[3]);
                    reinterpret_cast<int4 *>(it.z_out)[i] = zz;
                }
                if (it.a_out && i >= it.phase && ((i - it.phase) & 1) == 0) {
                    uint32_t packed = 0;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        int32_t q = clamp32(rs32(z[c], it.shift), -16, 15);
                        packed |= ((uint32_t)q & 0xFFu) << (8 * c);
                    }
                    reinterpret_cast<uint32_t *>(it.a_out)[(i - it.phase) >> 1] = packed;
                }
            }
        }
    }
}

// ----------------------------------------------------------------------- AEQ --

__device__ __forceinline__ uint32_t aeq_load(const AeqItem &it, int64_t i, int *err) {
    uint32_t w;
    if (i < 0) {
        w = it.hist_in ? reinterpret_cast<const uint32_t *>(it.hist_in)[16 + i] : 0u;
    } else {
        w = (uint64_t)i < it.m ? reinterpret_cast<const uint32_t *>(it.a)[i] : 0u;
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

__global__ __launch_bounds__(64) void aeq_fnt_kernel(const AeqItem *items, AeqItem single,
                                                     int *err) {
    using FF = Field<16>;
    const AeqItem it = items ? items[blockIdx.x] : single;
    const int lane = threadIdx.x;
    const int pos = lane & 31, half = lane >> 5;   // half 0: high digit, half 1: low digit
    const int s1 = lane >> 4, kk = lane & 15;       // gradient / tap-state ownership

    __shared__ int16_t tapl[256];                   // [S1][S2][k]
    __shared__ uint32_t epsw[16];                   // bytes [S2][j], eps of the block
    __shared__ uint32_t winw[36];                   // bytes [S1][32] window + zero pad

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

    // tap-digit spectra: W[f] = FNT32(digit_half(w_f) * 32^-1) at bin bitrev(pos)
    uint32_t W[16];
    auto transform_taps = [&]() {
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) tapl[(s1 * 4 + s2) * 16 + kk] = (int16_t)w[s2];
        __syncthreads();
#pragma unroll
        for (int f = 0; f < 16; ++f) {
            int32_t tv = (int32_t)tapl[f * 16 + (pos & 15)];
            tv = pos < 16 ? tv : 0;                 // zero padding 16 -> 32
            W[f] = fwd_xlane<16, 5, false>(tap_digit(tv, half), lane);
        }
        __syncthreads();
    };
    transform_taps();

    const int64_t nblocks = (int64_t)((M + 15) / 16);
    const int c2 = it.const_unit * it.const_unit;
    // lane pos holds window symbol 16 b - 16 + pos (both halves alike)
    uint32_t win = aeq_load(it, -16 + pos, err);

    for (int64_t b = 0; b < nblocks; ++b) {
        // prefetch the next block's 16 new symbols
        uint32_t nxt = pos >= 16 ? aeq_load(it, 16 * b + pos, err) : 0u;

        // input spectra: lanes 0-31 stream 0 / 2, lanes 32-63 stream 1 / 3
        int r01 = half ? sbyte(win, 1) : sbyte(win, 0);
        int r23 = half ? sbyte(win, 3) : sbyte(win, 2);
        uint32_t A01 = fwd_xlane<16, 5, false>(FF::from_int(r01), lane);
        uint32_t A23 = fwd_xlane<16, 5, false>(FF::from_int(r23), lane);
        uint32_t A01x = (uint32_t)__shfl_xor((int)A01, 32);
        uint32_t A23x = (uint32_t)__shfl_xor((int)A23, 32);
        uint32_t A[4];
        A[0] = half ? A01x : A01;
        A[1] = half ? A01 : A01x;
        A[2] = half ? A23x : A23;
        A[3] = half ? A23 : A23x;

        // Fermat-domain 4x4 MIMO: per output stream and polarisation pair, the
        // two input streams are summed before one inverse transform (Eq. (5)
        // holds for the pair: 2 * 16 taps * 64 * 16 = 32768 = (F - 1) / 2)
        int32_t t[4];
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
            uint32_t yx = FF::add(FF::mul(A[0], W[0 * 4 + s2]), FF::mul(A[1], W[1 * 4 + s2]));
            uint32_t yy = FF::add(FF::mul(A[2], W[2 * 4 + s2]), FF::mul(A[3], W[3 * 4 + s2]));
            yx = inv_xlane<16, 5, false>(yx, lane);
            yy = inv_xlane<16, 5, false>(yy, lane);
            t[s2] = FF::lift(yx) + FF::lift(yy);
        }
        // recombine the digit groups: y = 2^7 * (high-digit conv) + (low-digit conv)
        int32_t yh[4];
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
            int32_t lo = __shfl_xor(t[s2], 32);
            int32_t y = 128 * t[s2] + lo;
            yh[s2] = (int32_t)clamp64(rs64((int64_t)y, it.out_shift), -32768, 32767);
        }
        const int64_t m = 16 * b + (pos - 16);
        const bool outlane = half == 0 && pos >= 16;
        const bool valid = outlane && (uint64_t)m < M;
        if (valid) {
            uint2 o;
            o.x = ((uint32_t)yh[0] & 0xFFFFu) | ((uint32_t)yh[1] << 16);
            o.y = ((uint32_t)yh[2] & 0xFFFFu) | ((uint32_t)yh[3] << 16);
            reinterpret_cast<uint2 *>(it.out)[m] = o;
        }
        if (it.update_enable) {
            // RDE error per polarisation and the 8-bit error terms eps_S2
            uint32_t epack = 0;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                int64_t yi = yh[2 * p], yq = yh[2 * p + 1];
                int64_t r2 = yi * yi + yq * yq;
                int64_t R2 = r2 < 6LL * c2 ? 2LL * c2 : (r2 < 14LL * c2 ? 10LL * c2 : 18LL * c2);
                int64_t e = R2 - r2;
                int32_t ei = (int32_t)clamp64(rs64(e * yi, it.err_shift), -128, 127);
                int32_t eq = (int32_t)clamp64(rs64(e * yq, it.err_shift), -128, 127);
                epack |= ((uint32_t)ei & 0xFFu) << (16 * p);
                epack |= ((uint32_t)eq & 0xFFu) << (16 * p + 8);
            }
            if (!valid) epack = 0u;
            // stage eps (stream-major bytes) and the window (stream-major bytes)
            if (outlane) {
                uint8_t *eb = reinterpret_cast<uint8_t *>(epsw);
#pragma unroll
                for (int c = 0; c < 4; ++c) eb[c * 16 + (pos - 16)] = (uint8_t)(epack >> (8 * c));
            }
            if (half == 0) {
                uint8_t *wb = reinterpret_cast<uint8_t *>(winw);
#pragma unroll
                for (int c = 0; c < 4; ++c) wb[c * 32 + pos] = (uint8_t)(win >> (8 * c));
            }
            __syncthreads();
            // G[S1][S2][k] = sum_j eps_S2[j] * a_S1[16 b + j - k], as 4-byte dot products
            const int off = s1 * 32 + 16 - kk;          // byte offset of a_S1[16 b - k]
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
                w[s2] = clamp32(w[s2] + (int32_t)rs64((int64_t)g, it.mu_shift), -8192, 8191);
            }
            transform_taps();
        }
        // slide the window by 16 symbols
        uint32_t slid = (uint32_t)__shfl((int)win, (lane & 32) | ((pos + 16) & 31));
        win = pos < 16 ? slid : nxt;
    }
    aeq_finish(it, lane, w, err);
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
            reinterpret_cast<uint2 *>(it.out)[m] = o;
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
                w[s2] = clamp32(w[s2] + (int32_t)rs64((int64_t)g, it.mu_shift), -8192, 8191);
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

hipError_t launch_transform(const uint32_t *x, uint32_t *X, size_t batch, int t, int log2n,
                            int alpha_kind, bool inverse, int *err, hipStream_t s) {
    const uint64_t total = (uint64_t)batch << log2n;
    if (total == 0) return hipSuccess;
    const unsigned threads = 256;
    const unsigned grid = (unsigned)((total + threads - 1) / threads);
#define FNT_LAUNCH(Q, L, S)                                                                   \
    do {                                                                                      \
        if (inverse)                                                                          \
            fnt_transform_kernel<Q, L, S, true><<<grid, threads, 0, s>>>(x, X, total, err);  \
        else                                                                                  \
            fnt_transform_kernel<Q, L, S, false><<<grid, threads, 0, s>>>(x, X, total, err); \
    } while (0)
    if (t == 2 && log2n == 3 && alpha_kind == FNT_ALPHA_2) FNT_LAUNCH(4, 3, false);
    else if (t == 4 && log2n == 5 && alpha_kind == FNT_ALPHA_2) FNT_LAUNCH(16, 5, false);
    else if (t == 4 && log2n == 6 && alpha_kind == FNT_ALPHA_SQRT2) FNT_LAUNCH(16, 6, true);
    else return hipErrorInvalidValue;
#undef FNT_LAUNCH
    return hipGetLastError();
}

hipError_t launch_cdc(const CdcItem *items, int nitems, const CdcItem &single,
                      uint64_t total_blocks, int waves_per_group, int blocks_per_wave,
                      bool with_z, int *err, hipStream_t s) {
    if (total_blocks == 0) return hipSuccess;
    if (waves_per_group < 1 || waves_per_group > 4 || blocks_per_wave < 1)
        return hipErrorInvalidValue;
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

hipError_t launch_aeq(const AeqItem *items, int nitems, const AeqItem &single, int variant,
                      int *err, hipStream_t s) {
    const int grid = items ? nitems : 1;
    if (grid <= 0) return hipSuccess;
    if (variant == 0)
        aeq_fnt_kernel<<<grid, 64, 0, s>>>(items, single, err);
    else
        aeq_direct_kernel<<<grid, 64, 0, s>>>(items, single, err);
    return hipGetLastError();
}

}  // namespace fnti
