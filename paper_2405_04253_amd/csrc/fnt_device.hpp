// Device-side arithmetic in Z_F, F = 2^Q + 1 (a Fermat number, FNT section of
// the paper): canonical residues, loose residues modulo 65537, lane exchanges.
//
// Residues are uint32 in canonical form [0, F).  For Q = 16 (F = 65537) all
// reductions use 2^16 = -1 (mod F): a 32-bit value h*2^16 + l reduces to l - h.
// Multiplication by a power of the radix is a shift (alpha = 2) or a shift plus
// one multiply by 2^12 - 2^4 (alpha = sqrt 2), never a general product.

#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fntd {

template <int Q>
struct Field {
    static constexpr uint32_t F = (1u << Q) + 1u;

    // Reduce any uint32 to [0, F).
    static __device__ __forceinline__ uint32_t red(uint32_t x) {
        if constexpr (Q == 16) {
            int32_t r = (int32_t)(x & 0xFFFFu) - (int32_t)(x >> 16);
            return r < 0 ? (uint32_t)(r + (int32_t)F) : (uint32_t)r;
        } else {
            return x % F;
        }
    }
    // Signed integer with |v| < 2^31 - F to [0, F).
    static __device__ __forceinline__ uint32_t from_int(int32_t v) {
        if constexpr (Q == 16) {
            // v = h*2^16 + l with l in [0, 65535], h signed: v == l - h (mod F)
            int32_t r = (int32_t)((uint32_t)v & 0xFFFFu) - (v >> 16);  // in [-32767, 98303]
            r = r < 0 ? r + (int32_t)F : r;
            return r >= (int32_t)F ? (uint32_t)(r - (int32_t)F) : (uint32_t)r;
        } else {
            int32_t r = v % (int32_t)F;
            return (uint32_t)(r < 0 ? r + (int32_t)F : r);
        }
    }
    static __device__ __forceinline__ uint32_t add(uint32_t a, uint32_t b) {
        uint32_t s = a + b;
        return s >= F ? s - F : s;
    }
    static __device__ __forceinline__ uint32_t sub(uint32_t a, uint32_t b) {
        return a >= b ? a - b : a + F - b;
    }
    static __device__ __forceinline__ uint32_t neg(uint32_t a) { return a ? F - a : 0u; }
    // a * b for canonical a, b.
    static __device__ __forceinline__ uint32_t mul(uint32_t a, uint32_t b) {
        if constexpr (Q == 16) {
            uint64_t p = (uint64_t)a * b;             // <= 2^32
            uint32_t lo = (uint32_t)p, hi = (uint32_t)(p >> 32);
            uint32_t r = red(lo) + hi;                 // 2^32 == 1 (mod F)
            return r >= F ? r - F : r;
        } else {
            return (a * b) % F;
        }
    }
    // a * 2^e for canonical a, 0 <= e < 2Q (2^Q == -1).
    static __device__ __forceinline__ uint32_t mulpow2(uint32_t a, int e) {
        bool negate = e >= Q;
        int s = negate ? e - Q : e;
        uint32_t r;
        if constexpr (Q == 16) {
            r = red(a << s);                           // a <= 2^16, s <= 15: fits 32 bits
        } else {
            r = (a << s) % F;
        }
        return negate ? neg(r) : r;
    }
    // a * 2^(Q/4) * (2^(Q/2) - 1), the square root of 2 (Q >= 4).
    static __device__ __forceinline__ uint32_t mulsqrt2(uint32_t a) {
        constexpr uint32_t R = (1u << (3 * Q / 4)) - (1u << (Q / 4));
        if constexpr (Q == 16) {
            return red(a * R);                         // a * 4080 < 2^28
        } else {
            return (a * R) % F;
        }
    }
    // a * alpha^e, alpha = 2 (SQRT2 = false, 0 <= e < 2Q) or sqrt 2 (0 <= e < 4Q).
    template <bool SQRT2>
    static __device__ __forceinline__ uint32_t mul_radix_pow(uint32_t a, int e) {
        if constexpr (SQRT2) {
            uint32_t r = mulpow2(a, e >> 1);
            return (e & 1) ? mulsqrt2(r) : r;
        } else {
            return mulpow2(a, e);
        }
    }
    // Centred lift of a canonical residue to [-(F-1)/2, (F-1)/2].
    static __device__ __forceinline__ int32_t lift(uint32_t r) {
        return r > (F - 1) / 2 ? (int32_t)r - (int32_t)F : (int32_t)r;
    }
};

__device__ __forceinline__ int bitrev(int v, int bits) {
    return (int)(__brev((uint32_t)v) >> (32 - bits));
}

// Round half up then drop s bits (s >= 0), on 64-bit signed values.
__device__ __forceinline__ int64_t rs64(int64_t v, int s) {
    return s > 0 ? ((v + ((int64_t)1 << (s - 1))) >> s) : v;
}
__device__ __forceinline__ int32_t rs32(int32_t v, int s) {
    return s > 0 ? (int32_t)(((int64_t)v + ((int64_t)1 << (s - 1))) >> s) : v;
}
// rs32 in 32-bit arithmetic, given the rounding term r = 2^(s-1) (0 for s = 0)
// and |v| + r < 2^31.
__device__ __forceinline__ int32_t rs32r(int32_t v, int s, int32_t r) { return (v + r) >> s; }
__device__ __forceinline__ int64_t clamp64(int64_t v, int64_t lo, int64_t hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}
__device__ __forceinline__ int32_t clamp32(int32_t v, int32_t lo, int32_t hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

// ---------------------------------------------------------------------------
// Lazy arithmetic modulo F4 = 65537 on signed int32 ("loose residues").
//
// A loose residue is any int32 congruent to the value; callers keep the bounds
// stated at each use.  The only reduction is inside mulmod: for |v|, |c| < 2^23
// the 48-bit product v*c = hi*2^32 + lo (lo unsigned) is congruent to
// hi + lo[15:0] - lo[31:16] because 2^32 == 1 and 2^16 == -1 (mod 65537); the
// result has magnitude < 2^16 + 2^14.  The sign-extension idiom makes the
// compiler emit v_mul_i32_i24 / v_mul_hi_i32_i24 and SDWA word selects.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t sext24(int32_t v) { return (v << 8) >> 8; }

__device__ __forceinline__ int32_t mulmod(int32_t v, int32_t c) {
    int64_t p = (int64_t)sext24(v) * (int64_t)sext24(c);
    uint32_t lo = (uint32_t)p;
    int32_t hi = (int32_t)(p >> 32);
    return hi + (int32_t)(lo & 0xFFFFu) - (int32_t)(lo >> 16);
}

// A twiddle constant the compiler may not look into: powers of two would
// otherwise be strength-reduced from the 24-bit multiply of mulmod into a
// longer 64-bit shift sequence.  Non-volatile, so it is still hoisted.
__device__ __forceinline__ int32_t opq(int32_t v) {
    __asm__("" : "+v"(v));
    return v;
}

// Per-lane select (a where c, else b) -> v_cndmask_b32.
__device__ __forceinline__ int32_t blend(bool c, int32_t a, int32_t b) { return c ? a : b; }

// Centred representative in [-32768, 32768] of a loose residue (any int32).
__device__ __forceinline__ int32_t lift_loose(int32_t r) {
    int32_t f = (int32_t)((uint32_t)r & 0xFFFFu) - (r >> 16);   // in [-32767, 98303]
    f = f > 32768 ? f - 65537 : f;
    return f < -32768 ? f + 65537 : f;
}

// Lane exchange with lane ^ X inside a wave64 (DPP where one exists, else
// ds_swizzle inside 32-lane groups, else ds_bpermute).
template <int X>
__device__ __forceinline__ int32_t xor_lane(int32_t v) {
    // update_dpp with old = 0 and bound_ctrl: every lane has a partner here, and
    // the form lets the compiler fold the move into the consuming add / sub
    if constexpr (X == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true);   // quad_perm 1,0,3,2
    else if constexpr (X == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true);  // quad_perm 2,3,0,1
    else if constexpr (X == 8) return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, true); // row_ror:8
    else if constexpr (X == 4 || X == 16) return __builtin_amdgcn_ds_swizzle(v, (X << 10) | 0x1F);
    else return __shfl_xor(v, X);
}

// Lane order inside a transform group of up to 16 lanes.  Lanes with bit 2 set
// hold position l ^ 3, so the partner at position distance 4 is the DPP
// row_half_mirror lane (l ^ 7) and every in-row exchange of a transform is a
// DPP move (distance 1, 2: quad_perm; 4: row_half_mirror; 8: row_ror).
__device__ __forceinline__ int lane_pos(int l) { return (l & 4) ? (l ^ 3) : l; }
template <int X>
__device__ __forceinline__ int32_t xor_pos(int32_t v) {
    if constexpr (X == 4) return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true);  // row_half_mirror
    return xor_lane<X>(v);
}

// Global-address-space view of a device pointer.  Loads and stores through it
// are global_* instructions, which count only against the vector-memory
// counter; through a generic pointer they are flat_* instructions, which also
// count against the LDS counter, so every wait for an LDS result would wait for
// them as well.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gptr(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

// Range-violation bits latched into the per-device flag.
// RANGE_STALL is not a range violation: a bounded wait of the fused kernel gave
// up (its outputs are then unspecified).
enum : int { RANGE_SAMPLE = 1, RANGE_TAP = 2, RANGE_RESIDUE = 4, RANGE_SYMBOL = 8, RANGE_STALL = 16 };

}  // namespace fntd
