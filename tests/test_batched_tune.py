"""Host-side tests of the batched launch shape and the autotuners' cache (no GPU needed).

bsk_batched_shape reports the lanes, rows per work unit and orders per pass that a
batched call would launch with; the descriptors it plans from carry placeholder
addresses that are never dereferenced."""
import math
import os

import pytest

from paper_1107_4617_amd import _lib, batched_shape, tune_cache_clear, tune_cache_load, tune_cache_save


def _folded(N):
    return N // 2 + 1 if N % 2 == 0 else (N + 1) // 2


def _n0(sigma, T=255.0):
    return math.ceil((2 * T / (math.pi * sigma)) ** 2)


def _default_chunk(K, sizes=(16, 8, 12)):
    # the pass size with the lowest estimated cost, as the library picks it (ties keep the
    # earlier size: the full pass, its half, then 12 orders)
    cost = lambda kc: ((K + kc - 1) // kc) * (kc + 5.0 + 0.1 * kc)  # noqa: E731
    best = sizes[0]
    for kc in sizes[1:]:
        if cost(kc) < cost(best):
            best = kc
    return best


def _rb(r):
    return r.bit_length()


def _kb(K):
    return (K - 1).bit_length()


SHAPES = [(300, 200), (64, 900), (1500, 1200), (129, 128)]
RADII = [3, 20, 25, 9]
SIGMAS = [40.0, 12.0, 30.0, 55.0]


@pytest.fixture
def clean_cache():
    tune_cache_clear()
    yield
    tune_cache_clear()


def test_default_shape(clean_cache):
    block, rows, chunk = batched_shape(SHAPES, RADII, SIGMAS)
    assert block == 256
    assert rows == [min(96, h) for h, _ in SHAPES]
    assert chunk == [_default_chunk(_folded(_n0(s))) for s in SIGMAS]


def test_options_fix_the_shape(clean_cache):
    block, rows, chunk = batched_shape(SHAPES, RADII, SIGMAS, strip_h=40, order_chunk=8)
    assert block == 256 and rows == [min(40, h) for h, _ in SHAPES] and chunk == [8] * 4
    block, rows, chunk = batched_shape(SHAPES, RADII, SIGMAS, block=512)
    assert block == 512 and set(chunk) <= {8, 4}
    assert batched_shape(SHAPES, RADII, SIGMAS, order_chunk=12)[2] == [12] * 4
    with pytest.raises(_lib.BskError):
        batched_shape(SHAPES, RADII, SIGMAS, order_chunk=5)   # not a pass size of the kernel
    with pytest.raises(_lib.BskError):
        batched_shape(SHAPES, RADII, SIGMAS, block=512, order_chunk=12)   # 12 exists for 256 lanes only
    with pytest.raises(_lib.BskError):
        batched_shape(SHAPES, [300] + RADII[1:], SIGMAS, block=256)   # radius beyond a 256-lane strip


def test_cache_round_trip_applies_tuned_shapes(tmp_path, clean_cache):
    """A cache file written by hand in the tuner's format is loaded; batched plans then
    take the tuned rows and pass size for the images of the tuned bucket only, and the
    tuned lanes for batches whose largest radius falls in the tuned bucket; saving
    writes the same entries back; clearing restores the defaults."""
    K1 = _folded(_n0(SIGMAS[1]))
    rb1, kb1 = _rb(RADII[1]), _kb(K1)
    rbmax = max(_rb(r) for r in RADII)
    lines = [
        '{"batched_rb": %d, "kb": %d, "prec": 0, "block": 256, "S": 48, "kc": 8, "ms": 1.250000}' % (rb1, kb1),
        # the same bucket at another lane count: not used while the batch runs 256 lanes
        '{"batched_rb": %d, "kb": %d, "prec": 0, "block": 512, "S": 200, "kc": 4, "ms": 2.000000}' % (rb1, kb1),
        '{"batched_block_rb": %d, "prec": 0, "block": 256, "ms": 1.250000}' % rbmax,
        '{"rh": 20, "K": 16, "H": 4096, "W": 4096, "prec": 0, "block": 256, "S": 103, "kc": 16, "ms": 0.470000}',
    ]
    src = tmp_path / "tune.jsonl"
    src.write_text("\n".join(lines) + "\n")
    tune_cache_load(str(src))
    block, rows, chunk = batched_shape(SHAPES, RADII, SIGMAS)
    assert block == 256
    assert rows[1] == 48 and chunk[1] == 8
    for b in (0, 2, 3):
        assert (_rb(RADII[b]), _kb(_folded(_n0(SIGMAS[b])))) != (rb1, kb1)
        assert rows[b] == min(96, SHAPES[b][0])
        assert chunk[b] == _default_chunk(_folded(_n0(SIGMAS[b])))
    # explicit options still win over the table
    _, rows_o, chunk_o = batched_shape(SHAPES, RADII, SIGMAS, strip_h=64, order_chunk=16)
    assert rows_o[1] == 64 and chunk_o[1] == 16
    # a tuned lane count moves the whole batch to that kernel
    src2 = tmp_path / "tune2.jsonl"
    src2.write_text('{"batched_block_rb": %d, "prec": 0, "block": 512, "ms": 1.0}\n' % rbmax)
    tune_cache_load(str(src2))
    block, rows, chunk = batched_shape(SHAPES, RADII, SIGMAS)
    assert block == 512 and rows[1] == min(200, SHAPES[1][0]) and chunk[1] == 4
    # save writes every entry held; reloading it after a clear gives the same plans
    out = tmp_path / "saved.jsonl"
    tune_cache_save(str(out))
    saved = set(out.read_text().splitlines())
    assert set(lines[:2] + lines[3:]) <= saved
    assert '{"batched_block_rb": %d, "prec": 0, "block": 512, "ms": 1.000000}' % rbmax in saved
    tune_cache_clear()
    assert batched_shape(SHAPES, RADII, SIGMAS)[1][1] == min(96, SHAPES[1][0])
    tune_cache_load(str(out))
    assert batched_shape(SHAPES, RADII, SIGMAS) == (block, rows, chunk)


def test_cache_file_errors(tmp_path, clean_cache):
    with pytest.raises(_lib.BskError):
        tune_cache_load(str(tmp_path / "missing.jsonl"))
    with pytest.raises(_lib.BskError):
        tune_cache_save(str(tmp_path / "no_such_dir" / "x.jsonl"))
    # lines of no known kind are skipped
    junk = tmp_path / "junk.jsonl"
    junk.write_text("not json\n{\"other\": 1}\n")
    tune_cache_load(str(junk))
    assert batched_shape(SHAPES, RADII, SIGMAS)[1] == [min(96, h) for h, _ in SHAPES]
