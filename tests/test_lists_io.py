"""List files (april_lists_save / april_lists_load): round trips and damage.

The digest is pinned against Python's hashlib (an independent SHA-256), over
bodies whose lengths cover every 8-byte residue mod 64, including the two
padding cases (56 bytes left in the last block needs a whole extra block).
Damaged files (a flipped byte, a truncation, another magic or version, lists
that are not APRIL lists under a valid digest) must come back as
APRIL_E_CORRUPT, and missing files as APRIL_E_IO.
"""

import hashlib
import os

import numpy as np
import pytest

import synth
from paper_2307_01716_amd import april
from synth.grid import Grid
from synth.polygons import LATTICE

HEADER = 88
G6 = Grid(0.0, 0.0, 64 * (1 << 20) * LATTICE, 6)


def lists_with(n_a, n_f=0):
    """One object with n_a A intervals (and the first n_f of them as F)."""
    sA = np.arange(n_a, dtype=np.uint32) * 4 + 1
    eA = sA + 2
    return april.april_lists_from_arrays(G6, [0, n_a], sA, eA, [0, n_f], sA[:n_f], eA[:n_f])


def reseal(raw: bytes) -> bytes:
    body = raw[:-32]
    return body + hashlib.sha256(body).digest()


def test_digest_matches_hashlib_at_every_residue(tmp_path):
    seen = set()
    for n_a in range(0, 9):
        p = tmp_path / f"l{n_a}.apl"
        april.april_lists_save(lists_with(n_a), p)
        raw = p.read_bytes()
        body = raw[:-32]
        assert len(body) == HEADER + 16 * 2 + 8 * n_a
        assert raw[-32:] == hashlib.sha256(body).digest()
        seen.add(len(body) % 64)
    assert seen == set(range(0, 64, 8))
    assert not any(f.name.endswith(".tmp") for f in tmp_path.iterdir())


def test_round_trip_tiny(tmp_path):
    R, _, g = synth.configs.tiny()
    h = april.april_build_lists(g, R.xy, R.voff, april.STRICT)
    p = tmp_path / "r.apl"
    april.april_lists_save(h, p)
    back = april.april_lists_load(p)
    for a, b in zip(h.export(), back.export()):
        assert a.dtype == b.dtype and np.array_equal(a, b)
    i, j = h.info(), back.info()
    assert (i.n_objects, i.n_a, i.n_f, j.on_device) == (j.n_objects, j.n_a, j.n_f, -1)
    raw = p.read_bytes()
    assert raw[:8] == b"APRILLST"
    x0, y0, side = np.frombuffer(raw[16:40], np.float64)
    assert (x0, y0, side) == (g.x0, g.y0, g.side)
    assert int.from_bytes(raw[40:44], "little") == g.order
    # saving what was loaded writes the same bytes
    q = tmp_path / "again.apl"
    april.april_lists_save(back, q)
    assert q.read_bytes() == raw


def test_round_trip_partitioned_keeps_its_key(tmp_path):
    from paper_2307_01716_amd import partitioned
    R, S, _ = synth.configs.tiny(n=300)
    lay = synth.partitions.layout(R, S, 4, 10)
    h = partitioned.build_instances(lay, R, "r")
    p = tmp_path / "part.apl"
    april.april_lists_save(h, p)
    raw = p.read_bytes()
    assert int.from_bytes(raw[44:48], "little") == april.GRID_PARTITIONED
    assert int.from_bytes(raw[48:56], "little") != 0
    back = april.april_lists_load(p)
    q = tmp_path / "again.apl"
    april.april_lists_save(back, q)
    assert q.read_bytes() == raw


def test_empty_collection(tmp_path):
    L = april.april_lists_from_arrays(G6, [0], [], [], [0], [], [])
    p = tmp_path / "e.apl"
    april.april_lists_save(L, p)
    back = april.april_lists_load(p)
    assert back.info().n_objects == 0 and back.info().n_a == 0


def expect(code, fn, *a, **k):
    with pytest.raises(april.AprilError) as e:
        fn(*a, **k)
    assert e.value.code == code, str(e.value)


def test_damaged_files(tmp_path):
    good = tmp_path / "good.apl"
    april.april_lists_save(lists_with(5, 2), good)
    raw = good.read_bytes()
    bad = tmp_path / "bad.apl"

    def load(data, validate=True):
        bad.write_bytes(data)
        return april.april_lists_load(bad, validate)

    for k in (0, 9, 50, HEADER + 3, len(raw) - 40, len(raw) - 1):    # one flipped bit anywhere
        b = bytearray(raw)
        b[k] ^= 0x10
        expect(april.E_CORRUPT, load, bytes(b))
    expect(april.E_CORRUPT, load, raw[:-1])
    expect(april.E_CORRUPT, load, raw[:40])
    expect(april.E_CORRUPT, load, raw + b"\0")
    expect(april.E_CORRUPT, load, b"")
    expect(april.E_CORRUPT, load, reseal(b"APRILLSX" + raw[8:]))
    expect(april.E_CORRUPT, load, reseal(raw[:8] + (2).to_bytes(4, "little") + raw[12:]))
    # a count that does not fit the file, under a valid digest
    expect(april.E_CORRUPT, load, reseal(raw[:56] + (1 << 60).to_bytes(8, "little") + raw[64:]))
    expect(april.E_IO, april.april_lists_load, tmp_path / "missing.apl")
    expect(april.E_IO, april.april_lists_save, lists_with(1), tmp_path / "no" / "dir.apl")


def test_valid_digest_invalid_lists(tmp_path):
    p = tmp_path / "x.apl"
    april.april_lists_save(lists_with(5, 2), p)
    raw = bytearray(p.read_bytes())
    sA = HEADER + 16            # start_a follows off_a[2]
    # an A interval with start == end: not an APRIL list
    raw[sA:sA + 4] = (3).to_bytes(4, "little")
    data = reseal(bytes(raw))
    p.write_bytes(data)
    expect(april.E_CORRUPT, april.april_lists_load, p)
    assert april.april_lists_load(p, validate=False).info().n_a == 5
    # offsets that end past the intervals: rejected even without validation
    raw = bytearray(data)
    raw[HEADER + 8:HEADER + 16] = (6).to_bytes(8, "little")
    p.write_bytes(reseal(bytes(raw)))
    expect(april.E_CORRUPT, april.april_lists_load, p, False)
    # a grid that is not exact
    raw = bytearray(data)
    raw[40:44] = (17).to_bytes(4, "little")
    p.write_bytes(reseal(bytes(raw)))
    expect(april.E_CORRUPT, april.april_lists_load, p, False)


def test_save_rejects_null_and_keeps_old_file_on_failure(tmp_path):
    p = tmp_path / "keep.apl"
    april.april_lists_save(lists_with(2), p)
    before = p.read_bytes()
    os.chmod(tmp_path, 0o500)
    try:
        if os.access(tmp_path, os.W_OK):        # running as root: permissions do not bind
            pytest.skip("directory stays writable for this user")
        expect(april.E_IO, april.april_lists_save, lists_with(3), p)
    finally:
        os.chmod(tmp_path, 0o700)
    assert p.read_bytes() == before
