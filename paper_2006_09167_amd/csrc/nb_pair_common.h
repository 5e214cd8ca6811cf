// Device helpers shared by the pair kernels (forces, backward, list).
#pragma once

#include "nb_erfc_coeffs.h"
#include "nb_internal.h"

// Sum over the 8 consecutive lanes ii = 0..7 of a j-atom (row half): swap neighbours,
// swap pairs, then add the mirrored half row.  Each step adds two values in either order
// in the two lanes involved, so all eight lanes end with bitwise the same sum.
__device__ inline float dpp_sum8(float v) {
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0xB1, 0xF, 0xF, true));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x4E, 0xF, 0xF, true));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x141, 0xF, 0xF, true));
    return v;
}

// Periodic shift code (0..26) to its components in {-1, 0, 1}.
__device__ inline int shift_x(int code) { return code / 9 - 1; }
__device__ inline int shift_y(int code) { return (code / 3) % 3 - 1; }
__device__ inline int shift_z(int code) { return code % 3 - 1; }

// s L for s in {-1, 0, 1}: sign flip or zero applied to the bits of L (uniform operands,
// so this stays in scalar registers).
__device__ inline float shift_value(int s, float L) {
    int b = __builtin_bit_cast(int, L);
    asm("" : "+s"(b));   // opaque bits: the sign flip and the selection stay integer operations
    int v = s == 0 ? 0 : (s < 0 ? (b ^ (int)0x80000000u) : b);
    asm("" : "+s"(v));   // in a scalar register
    return __builtin_bit_cast(float, v);
}

// erfc(t) exp(t^2) = u P(u), u = 1/(1 + p t), t = beta r (coefficients fitted by
// fit_erfc.py; p_beta = p beta).
__device__ inline float erfcx_poly(float r, float p_beta) {
    const float u = __builtin_amdgcn_rcpf(fmaf(p_beta, r, 1.0f));   // 1 / (1 + p beta r)
    float p = NB_ERFC_C7;
    p = fmaf(p, u, NB_ERFC_C6);
    p = fmaf(p, u, NB_ERFC_C5);
    p = fmaf(p, u, NB_ERFC_C4);
    p = fmaf(p, u, NB_ERFC_C3);
    p = fmaf(p, u, NB_ERFC_C2);
    p = fmaf(p, u, NB_ERFC_C1);
    p = fmaf(p, u, NB_ERFC_C0);
    return u * p;
}

typedef float nb_f4 __attribute__((ext_vector_type(4)));

// A 16-byte store marked non-temporal: partial sums read once, later, by another kernel
// stream past the caches, so that they do not evict the coordinates.
__device__ inline void store_stream(float4* p, float x, float y, float z, float w) {
    const nb_f4 v = {x, y, z, w};
    __builtin_nontemporal_store(v, reinterpret_cast<nb_f4*>(p));
}
