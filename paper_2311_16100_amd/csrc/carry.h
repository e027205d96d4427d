// carry.h -- arithmetic of the packed LDS accumulator with wrap counters
// (gradient and HVP adjoint; see CarryScale in brick_kernels.hip).
//
// A complex contribution, rounded to integers (qr, qi) with |qr|, |qi| <
// 2^30, is added to a voxel's 64-bit word W as qr + 2^32 qi.  W then holds
// R + 2^32 I modulo 2^64 for the exact sums R, I.  With lo the low half of W
// read as a signed 32-bit number and H = (high half + [lo < 0]) mod 2^32
// read the same way, R = lo + 2^32 c_lo and I = H - c_lo + 2^32 c_hi, where
// c_lo and c_hi count the signed wraps of lo and of H.  A lane that adds to
// W receives the old word and, from it, the wraps its own addition made.
// The functions are host and device code, so that the accounting is tested
// on the CPU as well.
#pragma once
#include <stdint.h>

#ifndef CSG_HD
#include <hip/hip_runtime.h>
#define CSG_HD __host__ __device__ __forceinline__
#endif

// the 64-bit addend of (qr, qi)
CSG_HD unsigned long long carry_pack(int qr, int qi) {
    return (unsigned long long)(long long)qr + ((unsigned long long)(unsigned)qi << 32);
}

// Sign bit set unless lo and H both lie in [-2^30, 2^30), where no addend of
// at most 2^30 - 1 can wrap them.  One 64-bit addition tests both: lo + 2^30
// carries into the high half exactly when lo is in [-2^30, 0), so there the
// high half of the sum is H + 2^30.
CSG_HD uint32_t carry_may_wrap(unsigned long long old) {
    const unsigned long long t = old + 0x4000000040000000ull;
    return (uint32_t)t | (uint32_t)(t >> 32);
}

// the wraps (each -1, 0 or +1) of lo and of H made by adding (qr, qi) to the
// word whose value before the addition was `old`
CSG_HD void carry_wraps(unsigned long long old, int qr, int qi, int &dl, int &dh) {
    const int lo_old = (int)(uint32_t)old;
    const int lo_new = (int)((uint32_t)lo_old + (uint32_t)qr);
    dl = ((lo_old ^ lo_new) & (qr ^ lo_new)) < 0 ? (qr > 0 ? 1 : -1) : 0;
    const int h_old = (int)((uint32_t)(old >> 32) + (lo_old < 0 ? 1u : 0u));
    const long long h_new = (long long)h_old + qi + dl;
    dh = h_new > 0x7fffffffll ? 1 : (h_new < -0x80000000ll ? -1 : 0);
}

// The two counters of a voxel share one 32-bit word, c_lo + 2^16 c_hi: both
// stay below 2^15 in magnitude (a wrap needs 2^32 of sum, an addend is below
// 2^30, and a voxel receives at most 16 pixels of each of at most 1024
// images per work item, so at most 2^12 + 1 wraps), and the word's low half
// read as a signed 16-bit number is c_lo.
CSG_HD int carry_counter_step(int dl, int dh) { return dl + dh * 65536; }

CSG_HD void carry_counters(int w, int &c_lo, int &c_hi) {
    c_lo = (int)(short)(w & 0xFFFF);
    c_hi = (w - c_lo) >> 16;
}

// the exact sums of a word and its counters
CSG_HD void carry_decode(unsigned long long W, int c_lo, int c_hi, long long &R, long long &I) {
    const int lo = (int)(uint32_t)W;
    const int H = (int)((uint32_t)(W >> 32) + (lo < 0 ? 1u : 0u));
    R = (long long)lo + (long long)c_lo * 4294967296ll;
    I = (long long)H - c_lo + (long long)c_hi * 4294967296ll;
}
