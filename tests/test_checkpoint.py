"""Checkpoint files of a TT pair (the Picard iterate, Alg. 3.1), host side:
round trip, header, and every way a file can be refused."""
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import sys
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from paper_1906_06785_amd import sgtt
    return sgtt


def _pair(seed, dims=((5, 3, 40, 2, 4), (5, 3, 7, 3, 2))):
    g = np.random.default_rng(seed)
    out = []
    for n1, n2, n3, r1, r2 in dims:
        out.append((g.standard_normal((n1, r1)), g.standard_normal((r1, n2, r2)), g.standard_normal((n3, r2))))
    return tuple(out)


def test_round_trip_is_bit_exact(tmp_path):
    sg = _lib()
    x = _pair(1)
    f = str(tmp_path / "iterate.sgtt")
    sg.write_pair_host(f, x)
    assert not os.path.exists(f + ".tmp")
    assert sg.pair_file_info(f) == ((5, 3, 40, 2, 4), (5, 3, 7, 3, 2))
    y = sg.read_pair_host(f)
    for a, b in zip(x, y):
        for u, v in zip(a, b):
            assert u.shape == v.shape and np.array_equal(u, v)
    # larger capacities take the same file; ranks come from the file
    y = sg.read_pair_host(f, caps=((5, 3, 40, 8, 8), (5, 3, 7, 8, 8)))
    assert np.array_equal(y[0][2], x[0][2]) and np.array_equal(y[1][1], x[1][1])


def test_refusals(tmp_path):
    sg = _lib()
    x = _pair(2)
    f = str(tmp_path / "iterate.sgtt")
    sg.write_pair_host(f, x)
    raw = open(f, "rb").read()
    # ranks above the destination's capacity, sizes that differ
    with pytest.raises(sg.SgttError) as e:
        sg.read_pair_host(f, caps=((5, 3, 40, 1, 4), (5, 3, 7, 3, 2)))
    assert e.value.code == -4
    with pytest.raises(sg.SgttError) as e:
        sg.read_pair_host(f, caps=((5, 3, 41, 2, 4), (5, 3, 7, 3, 2)))
    assert e.value.code == -1
    # a flipped payload byte fails the hash; a cut file, a foreign file, a
    # missing file and an unwritable path are I/O errors
    bad = bytearray(raw)
    bad[200] ^= 0x40
    cases = {"flipped": bytes(bad), "cut": raw[:-9], "foreign": b"not a checkpoint" * 20}
    for name, data in cases.items():
        p = str(tmp_path / name)
        open(p, "wb").write(data)
        with pytest.raises(sg.SgttError) as e:
            sg.read_pair_host(p, caps=((5, 3, 40, 2, 4), (5, 3, 7, 3, 2)))
        assert e.value.code == -7, name
    with pytest.raises(sg.SgttError) as e:
        sg.pair_file_info(str(tmp_path / "missing"))
    assert e.value.code == -7
    with pytest.raises(sg.SgttError) as e:
        sg.write_pair_host(str(tmp_path / "no" / "such" / "dir"), x)
    assert e.value.code == -7
    # the header alone is checked by info (the hash needs the whole file)
    assert sg.pair_file_info(str(tmp_path / "flipped")) == ((5, 3, 40, 2, 4), (5, 3, 7, 3, 2))


def _net(seed, n=40, w=8):
    g = np.random.default_rng(seed)
    return g.standard_normal(w * n + w + w * w + w + n * w + n).astype(np.float32)


def test_network_file_round_trip_and_refusals(tmp_path):
    # parameter files of the learned correction's network
    sg = _lib()
    p = _net(3)
    f = str(tmp_path / "net.sgmlp")
    sg.write_mlp_host(f, 40, 8, p)
    assert not os.path.exists(f + ".tmp")
    assert sg.mlp_file_info(f) == (40, 8, p.size)
    assert np.array_equal(sg.read_mlp_host(f, 40, 8), p)
    raw = open(f, "rb").read()
    assert len(raw) == 8 + 4 + 8 + 8 + 4 * p.size + 8
    # another shape is refused as an invalid argument
    for n, w in ((41, 8), (40, 9)):
        with pytest.raises(sg.SgttError) as e:
            sg.read_mlp_host(f, n, w)
        assert e.value.code == -1
    # a flipped byte fails the hash; a cut, foreign, pair or missing file,
    # and a header whose parameter count does not fit its shape, are I/O errors
    bad = bytearray(raw)
    bad[100] ^= 0x01
    lie = bytearray(raw)
    lie[20] ^= 0x01   # the stored parameter count
    pair = str(tmp_path / "iterate.sgtt")
    sg.write_pair_host(pair, _pair(4))
    cases = {"flipped": bytes(bad), "cut": raw[:-5], "foreign": b"not a network" * 30, "count": bytes(lie)}
    for name, data in cases.items():
        g = str(tmp_path / f"{name}.sgmlp")
        open(g, "wb").write(data)
        with pytest.raises(sg.SgttError) as e:
            sg.read_mlp_host(g, 40, 8)
        assert e.value.code == -7, name
    for g in (pair, str(tmp_path / "missing.sgmlp")):
        with pytest.raises(sg.SgttError) as e:
            sg.read_mlp_host(g, 40, 8)
        assert e.value.code == -7
    with pytest.raises(sg.SgttError) as e:
        sg.write_mlp_host(str(tmp_path / "no" / "dir" / "net.sgmlp"), 40, 8, p)
    assert e.value.code == -7
