"""Pins of the oracle's random-number generator, electron wavelength and CTF.

* Philox4x32-10 against the published known-answer vectors
  (tests/golden/philox4x32_10_kat.txt).
* Rademacher probes (eq. (hutch), Sec. 3.2): values, balance and independence.
* Wavelength against textbook values (tests/golden/electron_wavelength.txt).
* CTF (Sec. 2.1 states only that it is real, radially symmetric and known):
  closed-form value at the origin, the bound |C| <= 1, and the zeros obtained
  by inverting chi(s) analytically.
"""
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        return [l.split() for l in f if l.strip() and not l.startswith("#")]


def test_philox_known_answers(orc):
    rows = _rows("philox4x32_10_kat.txt")
    assert len(rows) == 3
    for r in rows:
        vals = [int(x, 16) for x in r]
        out = orc.philox4x32_10(vals[0:4], vals[4:6])
        assert out.tolist() == vals[6:10]


def test_rademacher_values_balance_independence(orc):
    n = 1 << 20
    z1 = orc.rademacher(seed=7, probe=0, nvox=n)
    z2 = orc.rademacher(seed=7, probe=1, nvox=n)
    z3 = orc.rademacher(seed=8, probe=0, nvox=n)
    for z in (z1, z2, z3):
        assert set(np.unique(z).tolist()) == {-1.0, 1.0}
        assert abs(z.mean()) < 5.0 / math.sqrt(n)
    assert abs(np.mean(z1 * z2)) < 5.0 / math.sqrt(n)
    assert abs(np.mean(z1 * z3)) < 5.0 / math.sqrt(n)
    # neighbouring entries are independent too (no bit reuse between voxels)
    assert abs(np.mean(z1[1:] * z1[:-1])) < 5.0 / math.sqrt(n)
    # a prefix does not depend on how many entries are drawn
    assert np.array_equal(orc.rademacher(7, 0, 1000), z1[:1000])


def test_rademacher_bit_layout(orc):
    # The layout both implementations follow: entry k takes bit (k mod 128)
    # of the Philox block with counter (k // 128, probe_lo, probe_hi, 'RAD1').
    seed, probe = 0x1234_5678_9ABC, 3
    z = orc.rademacher(seed, probe, 300)
    for k in (0, 1, 31, 32, 127, 128, 129, 299):
        out = orc.philox4x32_10([k // 128, probe, 0, 0x52414431], [seed & 0xFFFFFFFF, seed >> 32])
        bit = (int(out[(k % 128) // 32]) >> (k % 32)) & 1
        assert z[k] == (-1.0 if bit else 1.0)


def test_wavelength_textbook(orc):
    for kv, lam in _rows("electron_wavelength.txt"):
        assert orc.wavelength_A(float(kv)) == pytest.approx(float(lam), rel=3e-3)


def test_ctf_origin_and_bound(orc):
    opt = orc.Optics()
    for df in (5000.0, 15000.0, 40000.0):
        # chi(0) = 0, so C(0) = -A
        assert orc.ctf(opt, 64, df, 0.0) == pytest.approx(-opt.amp_contrast, abs=1e-15)
        vals = [orc.ctf(opt, 64, df, float(k2)) for k2 in range(0, 32 * 32)]
        assert max(abs(v) for v in vals) <= 1.0 + 1e-15
        # underfocus: the phase term grows first, C moves from -A towards -1
        assert orc.ctf(opt, 256, df, 1.0) < -opt.amp_contrast
    assert orc.ctf(orc.NO_CTF, 64, 1e4, 100.0) == 1.0


@pytest.mark.parametrize("n_zero", [1, 2, 3])
def test_ctf_zeros_closed_form(orc, n_zero):
    # C = -(sqrt(1-A^2) sin chi + A cos chi) = -sin(chi + asin A) vanishes where
    # chi = n pi - asin A.  chi(s) = a s^2 - b s^4 is inverted analytically for
    # s^2, and the pixel size is chosen so that this s falls on |k| = 20 of a
    # 64 grid.
    A, kv, cs_mm, df = 0.1, 300.0, 2.7, 20000.0
    lam = orc.wavelength_A(kv)
    a = math.pi * lam * df
    b = 0.5 * math.pi * cs_mm * 1e7 * lam ** 3
    chi0 = n_zero * math.pi - math.asin(A)
    s2 = (a - math.sqrt(a * a - 4 * b * chi0)) / (2 * b)
    M, k = 64, 20
    pixel = k / (M * math.sqrt(s2))
    opt = orc.Optics(kv=kv, cs_mm=cs_mm, amp_contrast=A, pixel_A=pixel)
    assert abs(orc.ctf(opt, M, df, float(k * k))) < 1e-9
    # and an extremum half-way in phase: chi = (n - 1/2) pi - asin A gives C = -(+-1)
    chi1 = (n_zero - 0.5) * math.pi - math.asin(A)
    s2e = (a - math.sqrt(a * a - 4 * b * chi1)) / (2 * b)
    pixel_e = k / (M * math.sqrt(s2e))
    opt_e = orc.Optics(kv=kv, cs_mm=cs_mm, amp_contrast=A, pixel_A=pixel_e)
    assert abs(orc.ctf(opt_e, M, df, float(k * k))) == pytest.approx(1.0, abs=1e-9)


def test_ctf_spherical_aberration_only(orc):
    # df = 0, A = 0: C = -sin(-(pi/2) Cs lambda^3 s^4) = sin((pi/2) Cs lambda^3 s^4)
    opt = orc.Optics(amp_contrast=0.0)
    lam = orc.wavelength_A(300.0)
    M = 128
    for k2 in (100.0, 1000.0, 3000.0):
        s2 = k2 / (M * M)
        want = math.sin(0.5 * math.pi * 2.7e7 * lam ** 3 * s2 * s2)
        assert orc.ctf(opt, M, 0.0, k2) == pytest.approx(want, abs=1e-12)


def test_ctf_against_wave_aberration_in_angles(orc):
    # The phase written from the classical wave aberration instead of spatial
    # frequencies: a ray scattered by the angle theta = lambda s has the path
    # difference W(theta) = Cs theta^4 / 4 - df theta^2 / 2 (df > 0 meaning
    # underfocus here), and the phase is chi = -(2 pi / lambda) W.  Worked
    # example at 300 kV (lambda = 0.0196875 A), Cs = 2.7 mm, df = 0, s = 1/4 A^-1:
    #   theta = 4.9219e-3 rad, W = 6.75e6 A * theta^4 = 3.9612e-3 A,
    #   chi = -1.26420 rad, C = -(sqrt(0.99) sin chi + 0.1 cos chi) = 0.91840.
    # A wrong power of lambda or of s, or a wrong factor on the Cs term, moves
    # these values by far more than the tolerances.
    opt = orc.Optics()
    lam = orc.wavelength_A(300.0)
    assert lam == pytest.approx(0.0196875, abs=2e-7)
    M = 128
    assert orc.ctf(opt, M, 0.0, (0.25 * M) ** 2) == pytest.approx(0.91840, abs=2e-5)
    for df, s in ((0.0, 0.25), (0.0, 0.4), (15000.0, 0.25), (15000.0, 0.4), (32000.0, 0.11)):
        theta = lam * s
        W = 2.7e7 * theta ** 4 / 4.0 - df * theta ** 2 / 2.0
        chi = -2.0 * math.pi * W / lam
        want = -(math.sqrt(1.0 - 0.01) * math.sin(chi) + 0.1 * math.cos(chi))
        assert orc.ctf(opt, M, df, (s * M) ** 2) == pytest.approx(want, abs=1e-9)
