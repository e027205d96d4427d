"""The packed LDS accumulator of the gradient and HVP adjoint (carry.h),
compiled for the CPU: a voxel's 64-bit word plus its two wrap counters must
give back the exact integer sums of any sequence of addends below 2^30, in
particular sequences that wrap the 32-bit halves many times in either
direction; and an old word that passes the fast test must not wrap on any
such addend."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2311_16100_amd", "csrc")

HARNESS = r"""
#define CSG_HD static inline
#include "carry.h"
extern "C" {
// adds the n addends in order to one word, as the lanes of a kernel would
// one after another, and decodes the sums
void accumulate(const int *qr, const int *qi, long long n, long long *R, long long *I, int *wraps) {
    unsigned long long W = 0;
    int c_lo = 0, c_hi = 0, nw = 0;
    for (long long k = 0; k < n; ++k) {
        const unsigned long long old = W;
        W += carry_pack(qr[k], qi[k]);
        int dl, dh;
        carry_wraps(old, qr[k], qi[k], dl, dh);
        c_lo += dl;
        c_hi += dh;
        nw += (dl != 0) + (dh != 0);
    }
    carry_decode(W, c_lo, c_hi, *R, *I);
    *wraps = nw;
}
// the same with the two counters in one word, as the kernel keeps them
void accumulate_packed(const int *qr, const int *qi, long long n, long long *R, long long *I) {
    unsigned long long W = 0;
    int cw = 0;
    for (long long k = 0; k < n; ++k) {
        const unsigned long long old = W;
        W += carry_pack(qr[k], qi[k]);
        int dl, dh;
        carry_wraps(old, qr[k], qi[k], dl, dh);
        if (dl | dh) cw += carry_counter_step(dl, dh);
    }
    int c_lo, c_hi;
    carry_counters(cw, c_lo, c_hi);
    carry_decode(W, c_lo, c_hi, *R, *I);
}
unsigned may_wrap(unsigned long long old) { return carry_may_wrap(old); }
void wraps(unsigned long long old, int qr, int qi, int *dl, int *dh) { carry_wraps(old, qr, qi, *dl, *dh); }
}
"""


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    d = tmp_path_factory.mktemp("carry")
    src = d / "harness.cpp"
    src.write_text(HARNESS)
    so = d / "libcarry.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, str(src), "-o", str(so)], check=True)
    L = ctypes.CDLL(str(so))
    P = ctypes.POINTER
    L.accumulate.argtypes = [P(ctypes.c_int), P(ctypes.c_int), ctypes.c_longlong, P(ctypes.c_longlong),
                             P(ctypes.c_longlong), P(ctypes.c_int)]
    L.accumulate_packed.argtypes = [P(ctypes.c_int), P(ctypes.c_int), ctypes.c_longlong, P(ctypes.c_longlong),
                                    P(ctypes.c_longlong)]
    L.may_wrap.argtypes = [ctypes.c_ulonglong]
    L.may_wrap.restype = ctypes.c_uint
    L.wraps.argtypes = [ctypes.c_ulonglong, ctypes.c_int, ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int)]
    return L


def run(L, qr, qi):
    qr = np.ascontiguousarray(qr, dtype=np.int32)
    qi = np.ascontiguousarray(qi, dtype=np.int32)
    R, I, w = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int()
    L.accumulate(qr.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), qi.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                 len(qr), ctypes.byref(R), ctypes.byref(I), ctypes.byref(w))
    return R.value, I.value, w.value


LIM = 2 ** 30 - 1


def test_exact_sums_of_random_sequences(lib):
    rng = np.random.default_rng(5)
    for trial in range(300):
        n = int(rng.integers(1, 3000))
        lim = [LIM, 2 ** 29, 2 ** 20, 7][trial % 4]
        qr = rng.integers(-lim, lim + 1, n)
        qi = rng.integers(-lim, lim + 1, n)
        if trial % 3 == 1:  # one sign per component: the halves wrap in one direction only
            qr, qi = np.abs(qr) * rng.choice([-1, 1]), np.abs(qi) * rng.choice([-1, 1])
        R, I, _ = run(lib, qr, qi)
        assert R == int(qr.sum()) and I == int(qi.sum()), trial


def test_many_wraps_in_both_directions(lib):
    # thousands of wraps up, then back down through zero and beyond
    up = np.full(200_000, LIM)
    seq_r = np.concatenate([up, -up, -up[:1000]])
    seq_i = np.concatenate([-up, up, up[:777]])
    R, I, w = run(lib, seq_r, seq_i)
    assert (R, I) == (int(seq_r.sum()), int(seq_i.sum()))
    assert w > 100_000
    # alternating extremes around a large sum
    alt = np.tile([LIM, -LIM + 3], 50_000)
    R, I, _ = run(lib, alt, alt[::-1].copy())
    assert (R, I) == (int(alt.sum()), int(alt[::-1].sum()))


def test_counters_in_one_word(lib):
    """The kernel keeps both wrap counters in one 32-bit word; within the
    bound of one work item (16 pixels of each of 1024 images reach a voxel:
    16384 addends below 2^30, so at most 2^12 + 1 wraps of each half) the
    sums stay exact, in particular at that bound with addends of one sign."""
    rng = np.random.default_rng(7)
    cases = [(np.full(16384, LIM), np.full(16384, -LIM)), (np.full(16384, -LIM), np.full(16384, LIM))]
    for _ in range(60):
        n = int(rng.integers(1, 16385))
        cases.append((rng.integers(-LIM, LIM + 1, n) * rng.choice([-1, 1]), np.abs(rng.integers(-LIM, LIM + 1, n))))
    R, I = ctypes.c_longlong(), ctypes.c_longlong()
    for qr, qi in cases:
        qr = np.ascontiguousarray(qr, dtype=np.int32)
        qi = np.ascontiguousarray(qi, dtype=np.int32)
        lib.accumulate_packed(qr.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                              qi.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(qr), ctypes.byref(R), ctypes.byref(I))
        assert (R.value, I.value) == (int(qr.astype(np.int64).sum()), int(qi.astype(np.int64).sum()))


def _steps_to(total, last):
    """Addends below 2^30 in size that sum to `total` and end with `last`."""
    rest = total - last
    out = []
    while rest != 0:
        q = max(-LIM, min(LIM, rest))
        out.append(q)
        rest -= q
    return out + [last]


def test_sums_that_end_on_a_wrap_boundary(lib):
    """Every combination of a real sum just below, at and above each 32-bit
    boundary (so that lo ends negative or not) with an imaginary sum just
    below, at and above each boundary, reached by a last addend of either
    sign: the counters must catch the wraps of lo and of H = hi + [lo < 0]
    exactly at the boundary."""
    near = []
    for b in (2 ** 31, -2 ** 31, 2 ** 32 + 2 ** 31, -(2 ** 32) - 2 ** 31, 0):
        near += [b - 2, b - 1, b, b + 1]
    for R in near:
        for I in near:
            for last in (-3, 3, 1):
                qr = _steps_to(R, last)
                qi = _steps_to(I, -last)
                n = max(len(qr), len(qi))
                qr = [0] * (n - len(qr)) + qr
                qi = [0] * (n - len(qi)) + qi
                assert run(lib, qr, qi)[:2] == (R, I), (R, I, last)


def test_the_fast_test_admits_no_wrap(lib):
    """An old word whose halves pass the one-addition test cannot wrap on any
    addend below 2^30; near the test's bounds every case is tried."""
    rng = np.random.default_rng(6)
    edges = [-2 ** 31, -2 ** 30 - 1, -2 ** 30, -2 ** 30 + 1, -1, 0, 1, 2 ** 30 - 1, 2 ** 30, 2 ** 31 - 1]
    his = edges + list(rng.integers(-2 ** 31, 2 ** 31, 40))
    los = edges + list(rng.integers(-2 ** 31, 2 ** 31, 40))
    adds = [(LIM, LIM), (-LIM, -LIM), (LIM, -LIM), (-LIM, LIM), (1, -1), (0, 0)]
    dl, dh = ctypes.c_int(), ctypes.c_int()
    passed = 0
    for hi in his:
        for lo in los:
            old = ((int(hi) & 0xFFFFFFFF) << 32) | (int(lo) & 0xFFFFFFFF)
            H = ((int(hi) + (1 if lo < 0 else 0) + 2 ** 31) % 2 ** 32) - 2 ** 31
            fast = not (lib.may_wrap(old) & 0x80000000)
            assert fast == (-2 ** 30 <= lo < 2 ** 30 and -2 ** 30 <= H < 2 ** 30), (hi, lo)
            if fast:
                passed += 1
                for qr, qi in adds:
                    lib.wraps(old, qr, qi, ctypes.byref(dl), ctypes.byref(dh))
                    assert dl.value == 0 and dh.value == 0
    assert passed > 100
