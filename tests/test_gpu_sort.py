"""The radix sort primitive (ringo_sort_keys) on the GPU through the C ABI:
the conversion's LSD passes (Section 2.4 sorts the column copies) against a
stable sort by the same key bits (numpy's stable argsort), bit-exact, across
tile and run boundaries, digit counts, digit widths and key distributions."""
import contextlib
import sys

import numpy as np
import pytest

from paper_1503_07881_amd import ringo

pytestmark = pytest.mark.gpu

TILE = 2048  # 256 threads x 8 items: the scatter tile at the default schedule


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def expected(keys: np.ndarray, bits: int, digit: int | None = None) -> np.ndarray:
    """Stable sort by the low digit * ceil(bits / digit) bits (at most 64),
    digit being the schedule's digit width for that many keys unless given;
    higher bits ride along."""
    if digit is None:
        digit = ringo.tune_get(max(1, keys.size))[0]
    width = min(64, digit * ((bits + digit - 1) // digit))
    u = keys.view(np.uint64)
    k = u if width == 64 else u & np.uint64((1 << width) - 1)
    return keys[np.argsort(k, kind="stable")]


@contextlib.contextmanager
def digit_bits(bits):
    """Every size bucket's radix passes on `bits`-bit digits, restored after."""
    saved = [ringo.tune_get(1 << e) for e in range(63)]
    try:
        for e, (_, it, m) in enumerate(saved):
            ringo.tune_set(1 << e, bits, it, m)
        yield
    finally:
        for e, (d, it, m) in enumerate(saved):
            ringo.tune_set(1 << e, d, it, m)


def run(keys: np.ndarray, bits: int, dev) -> np.ndarray:
    import torch
    t = torch.from_numpy(np.ascontiguousarray(keys, dtype=np.int64)).to(dev)
    out = ringo.sort_keys(t, bits)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def keys_of(kind: str, n: int, bits: int, rng) -> np.ndarray:
    full = rng.integers(-(1 << 63), (1 << 63) - 1, n, dtype=np.int64, endpoint=True)
    width = 8 * ((bits + 7) // 8)
    low = np.uint64((1 << width) - 1) if width < 64 else np.uint64(~np.uint64(0))
    if kind == "uniform":
        return full
    if kind == "few":  # 17 distinct low parts, distinct high parts: stability shows
        low_vals = rng.integers(0, 1 << min(bits, 62), 17, dtype=np.int64)
        v = low_vals[rng.integers(0, 17, n)].view(np.uint64)
        hi = full.view(np.uint64) & ~low
        return (hi | (v & low)).view(np.int64)
    if kind == "equal":  # one low part for all: output = input order
        hi = full.view(np.uint64) & ~low
        return (hi | (np.uint64(0x5A5A5A5A5A5A5A5A) & low)).view(np.int64)
    if kind == "sorted":
        return expected(full, bits)
    if kind == "reverse":
        return expected(full, bits)[::-1].copy()
    raise ValueError(kind)


@pytest.mark.parametrize("n", [1, 2, TILE - 1, TILE, TILE + 1, 4 * TILE - 1, 4 * TILE + 1,
                               100_000, (1 << 20) + 3])
def test_sizes_across_tiles(cuda, n):
    rng = np.random.default_rng(1000 + n)
    for bits in (8, 64):
        say("sort_keys n", n, "bits", bits)
        keys = keys_of("uniform", n, bits, rng)
        assert np.array_equal(run(keys, bits, cuda), expected(keys, bits)), (n, bits)


@pytest.mark.parametrize("bits", [1, 7, 8, 9, 16, 22, 31, 32, 44, 63, 64])
def test_bit_widths(cuda, bits):
    rng = np.random.default_rng(2000 + bits)
    n = 3 * TILE * 8 + 11
    for kind in ("uniform", "few"):
        say("sort_keys bits", bits, kind)
        keys = keys_of(kind, n, bits, rng)
        assert np.array_equal(run(keys, bits, cuda), expected(keys, bits)), (bits, kind)


@pytest.mark.parametrize("kind", ["few", "equal", "sorted", "reverse"])
def test_distributions(cuda, kind):
    rng = np.random.default_rng(3000 + len(kind))
    for bits in (16, 40, 64):
        n = 250_001
        say("sort_keys", kind, "bits", bits)
        keys = keys_of(kind, n, bits, rng)
        got = run(keys, bits, cuda)
        assert np.array_equal(got, expected(keys, bits)), (kind, bits)
        if kind == "equal":
            assert np.array_equal(got, keys)  # a stable sort keeps the order


@pytest.mark.parametrize("n", [4096 * TILE - 1, 4096 * TILE, 4096 * TILE + 1])
def test_scan_paths_boundary(cuda, n):
    """Passes of at most 4096 tiles scan their counts in one kernel, larger
    ones in two: both sides of the switch."""
    rng = np.random.default_rng(5000 + n % 7)
    say("sort_keys scan boundary n", n)
    keys = keys_of("few", n, 24, rng)
    assert np.array_equal(run(keys, 24, cuda), expected(keys, 24))


def test_large(cuda):
    rng = np.random.default_rng(4000)
    n = (1 << 24) + 5
    say("sort_keys large n", n)
    keys = rng.integers(-(1 << 63), (1 << 63) - 1, n, dtype=np.int64, endpoint=True)
    assert np.array_equal(run(keys, 64, cuda), expected(keys, 64))


def test_empty_and_invalid(cuda):
    import torch
    e = torch.empty(0, dtype=torch.int64, device=cuda)
    assert ringo.sort_keys(e).numel() == 0
    t = torch.arange(10, dtype=torch.int64, device=cuda)
    with pytest.raises(ringo.RingoError):
        ringo.sort_keys_raw(t.data_ptr(), t.data_ptr() + 8, 4, 64, 0)  # overlapping
    with pytest.raises(ringo.RingoError):
        ringo.sort_keys(t, 0)


@pytest.mark.parametrize("digit", [9, 10, 11])
def test_digit_widths(cuda, digit):
    """Digits of 9 to 11 bits: ceil(bits / digit) passes, so the keys are
    ordered by the low digit * ceil(bits / digit) bits."""
    rng = np.random.default_rng(6000 + digit)
    with digit_bits(digit):
        for n in (1, TILE - 1, TILE + 1, 3 * TILE * 8 + 11, 300_007):
            for bits in (1, digit, digit + 1, 22, 33, 44, 63, 64):
                for kind in ("uniform", "few"):
                    say("sort_keys digit", digit, "n", n, "bits", bits, kind)
                    keys = keys_of(kind, n, bits, rng)
                    assert np.array_equal(run(keys, bits, cuda), expected(keys, bits, digit)), (n, bits, kind)
        # equal in the sorted bits (four digits): a stable sort keeps the order
        keys = keys_of("equal", 100_003, 4 * digit, rng)
        assert np.array_equal(run(keys, 4 * digit, cuda), keys)


@pytest.mark.parametrize("n", [4096 * TILE - 1, 4096 * TILE + 1])
def test_digit_widths_scan_paths(cuda, n):
    """Both scan kernels with 2048 digits per tile."""
    rng = np.random.default_rng(7000 + n % 7)
    with digit_bits(11):
        say("sort_keys 11-bit digits, scan boundary n", n)
        keys = keys_of("few", n, 30, rng)
        assert np.array_equal(run(keys, 30, cuda), expected(keys, 30, 11))


@contextlib.contextmanager
def schedule(digit, items):
    """Every size bucket on `digit`-bit digits and `items` keys per thread,
    restored after."""
    saved = [ringo.tune_get(1 << e) for e in range(63)]
    try:
        for e, (_, _, m) in enumerate(saved):
            ringo.tune_set(1 << e, digit, items, m)
        yield
    finally:
        for e, (d, it, m) in enumerate(saved):
            ringo.tune_set(1 << e, d, it, m)


PAIR_TILE = 2 * 256 * 16  # two halves of 256 threads x 16 keys


@pytest.mark.parametrize("digit", [8, 9])
def test_two_half_tiles(cuda, digit):
    """16 keys per thread with digits of at most 9 bits: the plain passes
    stage each 8192-key tile as two halves, ranked one after the other.
    Sizes around both tile sizes and a half, key widths, distributions."""
    rng = np.random.default_rng(8000 + digit)
    with schedule(digit, 16):
        for n in (1, 2, 4095, 4096, 4097, PAIR_TILE - 1, PAIR_TILE, PAIR_TILE + 1, 3 * PAIR_TILE + 17,
                  300_007):
            for bits in (1, digit, digit + 1, 17, 44, 64):
                for kind in ("uniform", "few"):
                    say("sort_keys two-half tiles digit", digit, "n", n, "bits", bits, kind)
                    keys = keys_of(kind, n, bits, rng)
                    assert np.array_equal(run(keys, bits, cuda), expected(keys, bits, digit)), (n, bits, kind)
        keys = keys_of("equal", 100_003, 3 * digit, rng)
        assert np.array_equal(run(keys, 3 * digit, cuda), keys)


@pytest.mark.parametrize("n", [4096 * PAIR_TILE - 1, 4096 * PAIR_TILE + 1])
def test_two_half_tiles_scan_paths(cuda, n):
    """Both scan kernels over 8192-key tiles."""
    rng = np.random.default_rng(9000 + n % 7)
    with schedule(9, 16):
        say("sort_keys two-half tiles, scan boundary n", n)
        keys = keys_of("few", n, 27, rng)
        assert np.array_equal(run(keys, 27, cuda), expected(keys, 27, 9))
