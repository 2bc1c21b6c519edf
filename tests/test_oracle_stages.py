"""Pins of the oracle's lossless stages (Sec. III-B on PFPL's pipeline,
Sec. IV-C): DIFFNB (delta + negabinary), BIT (bit transposition) and RZE
(zero elimination with a recursively compressed bitmap)."""
import numpy as np
import pytest


def negabinary_value(word: int, k: int) -> int:
    """Evaluate a negabinary digit string: sum of digit_j * (-2)^j."""
    return sum(((word >> j) & 1) * (-2) ** j for j in range(8 * k))


@pytest.mark.parametrize("k", [4, 8])
def test_negabinary_closed_forms(ref, k):
    table = {0: 0b0, 1: 0b1, -1: 0b11, 2: 0b110, -2: 0b10, 3: 0b111, -3: 0b1101,
             4: 0b100, -4: 0b1100, 6: 0b11010}
    for v, nb in table.items():
        # a one-word chunk: the delta from the implicit 0 is the value itself
        assert ref.diffnb(np.array([v]), k)[0] == nb
        assert negabinary_value(nb, k) == v


@pytest.mark.parametrize("k", [4, 8])
def test_diffnb_is_delta_then_negabinary(ref, k):
    rng = np.random.default_rng(k)
    lim = 2 ** 30 if k == 4 else 2 ** 60
    w = rng.integers(-lim, lim, 500)
    enc = ref.diffnb(w, k)
    mod = 2 ** (8 * k)
    prev = 0
    for i, v in enumerate(w.tolist()):
        d = (v - prev) % mod
        d = d - mod if d >= mod // 2 else d  # the signed delta modulo 2^(8k)
        assert negabinary_value(int(enc[i]) % mod, k) % mod == d % mod
        prev = v
    assert np.array_equal(ref.undiffnb(enc, k), w)


@pytest.mark.parametrize("k", [4, 8])
def test_bit_transposition(ref, k):
    m = 128
    for i, j in [(0, 0), (5, 3), (127, 8 * k - 1), (64, 17)]:
        words = np.zeros(m, np.uint64)
        words[i] = np.uint64(1) << np.uint64(j)
        data = b"".join(int(v).to_bytes(k, "little") for v in words.tolist())
        out = ref.bit(data, k)
        pos = j * m + i  # plane j, position i, planes lowest bit first
        expect = bytearray(m * k)
        expect[pos // 8] = 1 << (pos % 8)
        assert out == bytes(expect)
    rng = np.random.default_rng(9)
    data = rng.integers(0, 256, 64 * 3 * k).astype(np.uint8).tobytes()
    assert ref.unbit(ref.bit(data, k), k) == data


def test_rze_hand_example_with_one_bitmap_level(ref):
    data = bytearray(128)
    data[0] = 7
    data[100] = 9
    enc, pt = ref.rze(bytes(data), 1)
    assert not pt
    # bitmap: bits 0 and 100 -> 16 bytes [01, 0 x 11, 10, 0, 0, 0]; it is
    # longer than 8 bytes, so it is replaced by a 2-byte bitmap of the bytes
    # that differ from their predecessor (0, 1, 12, 13) plus those bytes
    assert enc == bytes([0x03, 0x30, 0x01, 0x00, 0x10, 0x00, 0x07, 0x09])
    assert ref.unrze(enc, 128, 1) == bytes(data)


def test_rze_small_example_word_size_4(ref):
    words = [0, 0, 5, 0] + [0] * 60
    data = b"".join(v.to_bytes(4, "little") for v in words)
    enc, pt = ref.rze(data, 4)
    # 64 words -> 8-byte bitmap (bit 2 set), stored as is, then the word
    assert enc == bytes([0x04] + [0] * 7) + (5).to_bytes(4, "little")
    assert ref.unrze(enc, 256, 4) == data


@pytest.mark.parametrize("w", [1, 4, 8])
@pytest.mark.parametrize("length", [64 * 8, 16384])
def test_rze_closed_forms_and_round_trips(ref, w, length):
    # all zero: only the top bitmap (all zero) survives
    enc, pt = ref.rze(bytes(length), w)
    items = length // w
    sizes = [(items + 7) // 8]
    while sizes[-1] > 8:
        sizes.append((sizes[-1] + 7) // 8)
    assert not pt and enc == bytes(sizes[-1])
    # incompressible: every word nonzero -> stored verbatim (passthrough)
    rng = np.random.default_rng(w + length)
    dense = rng.integers(1, 256, length).astype(np.uint8).tobytes()
    enc, pt = ref.rze(dense, w)
    assert pt and enc == dense
    for dens in (0.001, 0.05, 0.4):
        a = ((rng.random(length) < dens) * rng.integers(1, 256, length)).astype(np.uint8).tobytes()
        enc, pt = ref.rze(a, w)
        if not pt:
            assert len(enc) < length
            assert ref.unrze(enc, length, w) == a


def test_rze_rejects_bad_lengths(ref):
    data = bytearray(256)
    data[3] = 1
    enc, _ = ref.rze(bytes(data), 1)
    with pytest.raises(ref.OracleError):
        ref.unrze(enc + b"\x00", 256, 1)
    with pytest.raises(ref.OracleError):
        ref.unrze(enc[:-1], 256, 1)
