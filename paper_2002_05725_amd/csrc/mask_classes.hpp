// Row classes of QUAD masks, shared by the apply and gradient kernels.
//
// A thread owns the rows tid + (k << lane_bits) of a tile, k < 2^kb.  For each
// of the kb k bits a QUAD mask either flips it, has it in its Z string, or
// neither (flipped qubits are never in the Z string).  The class index has one
// base-3 digit per k bit (1 = flipped, 2 = in the Z string); within a class
// the source offset and the sign of every row are compile-time constants.
#pragma once

#include <utility>

#include "terms.hpp"

namespace syk {

// Bits b < kb whose base-3 digit of cls equals digit.
constexpr int class_bits(int cls, int kb, int digit)
{
    int r = 0;
    for (int b = 0; b < kb; ++b) {
        if (cls % 3 == digit) r |= 1 << b;
        cls /= 3;
    }
    return r;
}

constexpr int ipow3(int n) { return n == 0 ? 1 : 3 * ipow3(n - 1); }
constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

// Class of a QUAD mask for lane_bits lane bits and kb k bits.
inline int quad_class(uint32_t x, uint32_t zbase, int lane_bits, int kb)
{
    int cls = 0, p3 = 1;
    for (int b = 0; b < kb; ++b, p3 *= 3) {
        const uint32_t q = (uint32_t)(lane_bits + b);
        if ((x >> q) & 1u) cls += p3;
        else if ((zbase >> q) & 1u) cls += 2 * p3;
    }
    return cls;
}

// Groups of the apply kernel (three k bits): three QUAD masks that flip the
// same lane and tile qubits and J = 1 or 2 of the k bits, in all three ways.
// They read the same source rows.  Member j flips the k bits group_xk(J, j);
// a k bit b it does not flip is in its Z string when the flipped k bits above
// b plus the flipped qubits above the k bits (parity P) are odd in number.
// Group class GC = 2 (J - 1) + P.
constexpr int kQuadGroupClasses = 4;
constexpr int popc3(int v) { return (v & 1) + ((v >> 1) & 1) + ((v >> 2) & 1); }
constexpr int group_xk(int J, int j) { return J == 1 ? 1 << j : 7 ^ (1 << (2 - j)); }
constexpr int group_zk(int xk, int P)
{
    int z = 0;
    for (int b = 0; b < 3; ++b)
        if (!((xk >> b) & 1) && ((popc3(xk >> (b + 1)) + P) & 1)) z |= 1 << b;
    return z;
}
constexpr int group_member_class(int GC, int j)
{
    const int xk = group_xk(1 + (GC >> 1), j), zk = group_zk(xk, GC & 1);
    int cls = 0, p3 = 1;
    for (int b = 0; b < 3; ++b, p3 *= 3) cls += p3 * (((xk >> b) & 1) ? 1 : ((zk >> b) & 1) ? 2 : 0);
    return cls;
}
// The bits of p at the set bits of m, packed from bit 0 (three bits).
constexpr int pack_bits3(int p, int m)
{
    int r = 0, o = 0;
    for (int b = 0; b < 3; ++b)
        if ((m >> b) & 1) {
            if ((p >> b) & 1) r |= 1 << o;
            ++o;
        }
    return r;
}

// Calls f(std::integral_constant<int, I>{}) for every I of the sequence.
template <typename F, int... I>
__device__ __forceinline__ void for_each_class(F& f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}

// Sign flip by a word whose bit 31 is the sign to apply (other bits zero).
__device__ __forceinline__ double flip31(double x, uint32_t s)
{
    return __hiloint2double(__double2hiint(x) ^ (int)s, __double2loint(x));
}
__device__ __forceinline__ float flip31(float x, uint32_t s) { return __int_as_float(__float_as_int(x) ^ (int)s); }

}  // namespace syk
