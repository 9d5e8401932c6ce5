// bz_arith.hpp -- bit-sliced F_3 / F_7 arithmetic on 32-bit words (device and host).
//
// A vector of symbols is held as r bit planes (r = 2 for F_3, 3 for F_7): bit t
// of plane b is bit b of the natural binary expansion of symbol t (Sec. 2 of
// Hernando & Quintana-Orti, arXiv 2603.29942).  Natural encodings:
//   F_3: 0 = (0,0), 1 = (1,0), 2 = (0,1);   F_7: value = b0 + 2 b1 + 4 b2.
// Every function works on 32 symbols at once, one word per plane.  Inputs are
// canonical (no F_3 pattern (1,1), no F_7 pattern (1,1,1)); outputs are too.
// Padding positions hold zero in every plane and stay zero.
#pragma once
#include <stdint.h>

#ifndef BZ_HD
#define BZ_HD __host__ __device__ __forceinline__
#endif

namespace bz {

typedef uint32_t u32;

// ---------------------------------------------------------------- F_3
// a + b, Algorithm 3.  Bit 0 is a half adder; the carry out of bit 1 is 2+2 = 4
// = 1 (mod 3) and wraps to bit 0.  The listing combines that wrapped carry into
// s_0 with an `and`; that fails e.g. 2 + 2, so it is read as `xor` (with `or`
// the result is the same on canonical inputs).  The final step maps the
// pattern (1,1) = 3 to 0.  Nine boolean operations as in the paper.
BZ_HD void f3_add(u32 a0, u32 a1, u32 b0, u32 b1, u32 &s0, u32 &s1) {
    u32 c0 = a0 & b0;
    u32 c1 = a1 & b1;
    u32 t0 = a0 ^ b0 ^ c1;
    u32 t1 = a1 ^ b1 ^ c0;
    u32 t = t0 & t1;
    s0 = t0 ^ t;
    s1 = t1 ^ t;
}

// -x and 2x are the same map in F_3 (2 = -1): swap the planes (Sec. 4.2).
BZ_HD void f3_neg(u32 a0, u32 a1, u32 &s0, u32 &s1) { s0 = a1; s1 = a0; }

// nonzero mask of a + b, isometric addition for F_3 (Sec. 4.3): with c = a | b,
// a + b != 0 exactly where c_0 xor c_1 = 1.
BZ_HD u32 f3_iso_add(u32 a0, u32 a1, u32 b0, u32 b1) { return (a0 | b0) ^ (a1 | b1); }

// nonzero mask of a - b, isometric subtraction (Sec. 4.3): a != b somewhere in the planes.
BZ_HD u32 f3_iso_sub(u32 a0, u32 a1, u32 b0, u32 b1) { return (a0 ^ b0) | (a1 ^ b1); }

// ---------------------------------------------------------------- F_7
// a + b, Algorithm 4: a 3-bit ripple-carry sum, the carry out of bit 2 (8 = 1
// mod 7) added back at bit 0 (it cannot overflow again: a + b - 8 <= 6), then
// the pattern (1,1,1) = 7 mapped to 0.
BZ_HD void f7_add(u32 a0, u32 a1, u32 a2, u32 b0, u32 b1, u32 b2, u32 &s0, u32 &s1, u32 &s2) {
    u32 x0 = a0 ^ b0, c0 = a0 & b0;
    u32 x1 = a1 ^ b1 ^ c0, c1 = (a1 & b1) | (c0 & (a1 ^ b1));
    u32 x2 = a2 ^ b2 ^ c1, c2 = (a2 & b2) | (c1 & (a2 ^ b2));
    u32 e0 = x0 & c2;
    x0 ^= c2;
    u32 e1 = x1 & e0;
    x1 ^= e0;
    x2 ^= e1;
    u32 t = x0 & x1 & x2;
    s0 = x0 ^ t;
    s1 = x1 ^ t;
    s2 = x2 ^ t;
}

// 2x: circular shift of the expansion, bit i -> bit i+1, bit 2 -> bit 0 (Sec. 4.2).
BZ_HD void f7_double(u32 a0, u32 a1, u32 a2, u32 &s0, u32 &s1, u32 &s2) {
    s0 = a2; s1 = a0; s2 = a1;
}

// -x = 7 - x: the 3-bit complement, kept at 0 where x = 0 (masking also keeps
// the padding zero).
BZ_HD void f7_neg(u32 a0, u32 a1, u32 a2, u32 &s0, u32 &s1, u32 &s2) {
    u32 any = a0 | a1 | a2;
    s0 = ~a0 & any; s1 = ~a1 & any; s2 = ~a2 & any;
}

// nonzero mask of a + b, isometric addition for p = 2^r - 1 (Sec. 4.3):
// (OR_i xnor(a_i, b_i)) and (OR_i (a_i or b_i)).  Needs canonical inputs.
BZ_HD u32 f7_iso_add(u32 a0, u32 a1, u32 a2, u32 b0, u32 b1, u32 b2) {
    return ~((a0 ^ b0) & (a1 ^ b1) & (a2 ^ b2)) & (a0 | a1 | a2 | b0 | b1 | b2);
}

BZ_HD u32 f7_iso_sub(u32 a0, u32 a1, u32 a2, u32 b0, u32 b1, u32 b2) {
    return (a0 ^ b0) | (a1 ^ b1) | (a2 ^ b2);
}

// ---------------------------------------------------------------- scaled rows
// h * x for h in F_p^*, h = +-2^e: rotate by e, negate when h = p - 2^e.
template <int P>
BZ_HD void scale(int h, const u32 *x, u32 *y);

template <>
BZ_HD void scale<3>(int h, const u32 *x, u32 *y) {
    if (h == 1) { y[0] = x[0]; y[1] = x[1]; }
    else { y[0] = x[1]; y[1] = x[0]; }
}

template <>
BZ_HD void scale<7>(int h, const u32 *x, u32 *y) {
    // h -> (e, negate): 1:(0,0) 2:(1,0) 4:(2,0) 6:(0,1) 5:(1,1) 3:(2,1)
    int e = (h == 1 || h == 6) ? 0 : (h == 2 || h == 5) ? 1 : 2;
    bool neg = (h == 3 || h == 5 || h == 6);
    u32 r0 = x[0], r1 = x[1], r2 = x[2];
    for (int i = 0; i < e; i++) { u32 t = r2; r2 = r1; r1 = r0; r0 = t; }
    if (neg) { f7_neg(r0, r1, r2, y[0], y[1], y[2]); }
    else { y[0] = r0; y[1] = r1; y[2] = r2; }
}

// ---------------------------------------------------------------- compress
// The bits of x selected by a mask m, packed in order into the low bits: the
// parallel-suffix compress of Hacker's Delight (sec. 7-4).  The five move
// masks depend on m alone, so a mask shared by many words is planned once.
struct Compress32 {
    u32 mv[5];
};
BZ_HD Compress32 compress_plan(u32 m) {
    Compress32 c;
    u32 mk = ~m << 1;  // zeros of m to the right of each position, counted in parallel
    for (int i = 0; i < 5; i++) {
        u32 mp = mk ^ (mk << 1);
        mp ^= mp << 2;
        mp ^= mp << 4;
        mp ^= mp << 8;
        mp ^= mp << 16;  // parity of the zeros below each bit, per bit of the count
        const u32 mv = mp & m;
        c.mv[i] = mv;
        m = (m ^ mv) | (mv >> (1 << i));
        mk &= ~mp;
    }
    return c;
}
BZ_HD u32 compress_apply(u32 x, u32 m, const Compress32 &c) {
    x &= m;
#pragma unroll
    for (int i = 0; i < 5; i++) {
        const u32 t = x & c.mv[i];
        x = (x ^ t) | (t >> (1 << i));
    }
    return x;
}

// modular inverse in F_p^* (small tables)
BZ_HD int inv_mod(int P, int x) {
    if (P == 3) return x;  // 1 -> 1, 2 -> 2
    // F_7: 1->1 2->4 3->5 4->2 5->3 6->6
    return x == 1 ? 1 : x == 2 ? 4 : x == 3 ? 5 : x == 4 ? 2 : x == 5 ? 3 : 6;
}

}  // namespace bz
