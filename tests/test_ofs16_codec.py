"""Pins of the host model of the 16-bit offset words (tests/ofs16.py) against
facts of the formats themselves: FP16/BF16 bit patterns, the bit-14 flag
convention, exact pure phases, and the rounding bound on random states."""
import numpy as np
import pytest

import ofs16

P = dict(rho0_R=1.0, rho0_B=0.1, alpha_R=0.95, alpha_B=0.5)


def test_half_formats_known_bits():
    assert int(ofs16.f16_bits(np.float32(0.5))) == 0x3800
    assert int(ofs16.f16_bits(np.float32(-2.0))) == 0xC000
    assert int(ofs16.f16_bits(np.float32(2.0 ** -24))) == 0x0001   # smallest subnormal
    assert int(ofs16.bf16_bits(np.float32(1.0))) == 0x3F80
    # ties to even
    assert float(ofs16.bf16_value(ofs16.bf16_bits(np.float32(1.0 + 2.0 ** -8)))) == 1.0
    assert float(ofs16.bf16_value(ofs16.bf16_bits(np.float32(1.0 + 3 * 2.0 ** -8)))) == 1.0 + 2.0 ** -6
    assert float(ofs16.f16_value(ofs16.f16_bits(np.float32(1.0 + 2.0 ** -11)))) == 1.0


def test_bit14_is_clear_below_two():
    """Every finite FP16 value of magnitude below 2 has bit 14 clear, so the
    bit is free to carry the colour flag."""
    h = np.arange(65536, dtype=np.uint32)
    v = ofs16.f16_value(h).astype(np.float64)
    small = np.isfinite(v) & (np.abs(v) < 2.0)
    assert np.all((h[small] & 0x4000) == 0)
    assert np.all((h[np.isfinite(v) & (np.abs(v) >= 2.0)] & 0x4000) != 0)
    assert float(ofs16.ZMAX) == float(ofs16.f16_value(np.uint32(0x3FFF)))


def test_pure_phases_round_trip_exactly():
    fr, _ = ofs16.frefs(P)
    R = np.array([0.95] + [fr[ofs16.CLS[i]] for i in range(1, 9)], dtype=np.float32)[:, None]
    Z = np.zeros_like(R)
    for fmt in ("f16", "bf16"):
        w = ofs16.encode(R, Z, P, fmt)        # pure red: blue (the smaller) stored as 0
        assert np.all(w[2:] == 0x40000000)
        R2, B2 = ofs16.decode(w, P, fmt)
        assert np.array_equal(R2, R) and np.array_equal(B2, Z)
        w = ofs16.encode(Z, R, P, fmt)        # pure blue at the same f: red stored as 0
        assert np.all(w[2:] == 0)
        R2, B2 = ofs16.decode(w, P, fmt)
        assert np.array_equal(R2, Z) and np.array_equal(B2, R)


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_round_trip_within_bound(fmt):
    rng = np.random.default_rng(0)
    fr, _ = ofs16.frefs(P)
    n = 20000
    x = rng.uniform(0, 1, n)                    # red fraction, including extreme tails
    x = np.where(rng.uniform(size=n) < 0.3, x ** 12, x)
    f = np.empty((9, n))
    f[0] = rng.uniform(0.05, 0.95, n)
    for i in range(1, 9):
        f[i] = fr[ofs16.CLS[i]] * (1 + 0.02 * rng.standard_normal(n))
    R = x * f
    B = (1 - x) * f
    R[1:, :500] -= 2e-4                          # negative minority populations
    w = ofs16.encode(R, B, P, fmt)
    got = ofs16.decode_pair(w, P, fmt)
    ref = np.stack([R.astype(np.float32), B.astype(np.float32)]).astype(np.float64)
    err = np.abs(got - ref)
    assert np.all(err <= ofs16.rounding_bound(ref, P, fmt))
    # the minority colour keeps FP16 relative precision in its normal range
    # (unit 4 fref)
    s = np.minimum(np.abs(ref[0, 1:]), np.abs(ref[1, 1:]))
    frk = np.array([fr[ofs16.CLS[i]] for i in range(1, 9)])[:, None]
    normal = s > 2.0 ** -14 * 4 * frk
    sel_err = np.where(np.abs(ref[0, 1:]) <= np.abs(ref[1, 1:]), err[0, 1:], err[1, 1:])
    assert np.all(sel_err[normal] <= 2.0 ** -11 * s[normal] * (1 + 1e-6) + 2.0 ** -23 * frk.repeat(n, 1)[normal])


def test_pull_words_moves_each_word_once():
    ny, nx = 5, 7
    W = np.arange(10 * ny * nx, dtype=np.uint32).reshape(10, ny, nx)
    for walls in (False, True):
        out = ofs16.pull_words(W, walls)
        rows = slice(1, ny - 1) if walls else slice(0, ny)
        # rest-link words stay, word of link 8 (c = (1, 0)) comes from x - 1
        assert np.array_equal(out[0, rows], W[0, rows])
        assert np.array_equal(out[9, rows], np.roll(W[9], 1, axis=-1)[rows])
        if walls:
            # link 2 (c = (0, 1)) at the first fluid row bounces from link 6 of the same site
            assert np.array_equal(out[3, 1], W[7, 1])


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_signs_and_range_of_the_stored_colour(fmt):
    """The colour of smaller magnitude is stored with its sign; states with
    negative populations of either or both colours round-trip within the
    bound as long as one colour is below 8 fref in magnitude."""
    fr, _ = ofs16.frefs(P)
    rng = np.random.default_rng(1)
    n = 5000
    R = np.zeros((9, n))
    B = np.zeros((9, n))
    R[0], B[0] = 0.5, 0.05
    for i in range(1, 9):
        f = fr[ofs16.CLS[i]]
        R[i] = rng.uniform(-7.9, 7.9, n) * f
        B[i] = rng.uniform(-7.9, 7.9, n) * f
    ref = np.stack([R.astype(np.float32), B.astype(np.float32)]).astype(np.float64)
    got = ofs16.decode_pair(ofs16.encode(R, B, P, fmt), P, fmt)
    assert np.all(np.abs(got - ref) <= ofs16.rounding_bound(ref, P, fmt))
    w = ofs16.encode(R, B, P, fmt)
    blue_flag = (w[2:] >> 30) & 1
    assert np.array_equal(blue_flag.astype(bool), np.abs(ref[1, 1:]) < np.abs(ref[0, 1:]))
