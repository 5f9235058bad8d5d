"""Host-side checks of libesg (no GPU needed): exported symbols, status
strings, the index builder's output structure and determinism, and the
loader's rejection of malformed files."""
from __future__ import annotations

import os
import re
import shutil
import struct

import numpy as np
import pytest

import oracle
import synth
import paper_2504_04018_amd as esg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_exported():
    txt = open(os.path.join(ROOT, "include", "esg.h")).read()
    names = set(re.findall(r"^\s*(?:int32_t|void|const char\*)\s+(esg_\w+)\s*\(", txt, re.M))
    assert len(names) >= 9
    L = esg.lib()
    for n in names:
        assert hasattr(L, n), n
    assert names <= set(esg.SIGNATURES), names - set(esg.SIGNATURES)


def test_status_strings():
    for s in range(0, -9, -1):
        assert esg.status_str(s).startswith("ESG")
    assert "unknown" in esg.status_str(-99)


@pytest.fixture(scope="module")
def small_index(tmp_path_factory):
    w = synth.make_workload(0, n=3000, nq=0)
    d = tmp_path_factory.mktemp("cabi")
    path = str(d / "s.esgi")
    esg.build_index(w["X"], w["attr"].astype(np.float64), path, degree=12, leaf=100,
                    ef_construction=64)
    return w, path


def test_builder_structure(small_index):
    """Alg. 3 output: one graph per tree node with b-a >= leaf, neighbours
    inside the node, no self loops or repeats, degree <= R, rows packed,
    entry point inside the node, position order = attribute order."""
    w, path = small_index
    ix = oracle.read_index(path)
    assert np.array_equal(np.sort(w["attr"]), ix.attr)
    assert np.array_equal(ix.vec, w["X"][ix.ext_id])
    from tests.helpers import tree_nodes
    depth_seen = set()
    for t, h, a, b, g in tree_nodes(ix.n, ix.leaf):
        if not g:
            continue
        depth_seen.add(t)
        e = int(ix.ep[h])
        assert a <= e <= b
        rows = ix.adj[t, a:b + 1]
        valid = rows != oracle.NO_NODE
        # packed: no valid entry after a pad
        assert np.all(np.diff(valid.astype(int), axis=1) <= 0)
        vals = rows[valid].astype(np.int64)
        assert np.all((vals >= a) & (vals <= b))
        for i, row in enumerate(rows):
            rv = row[row != oracle.NO_NODE]
            assert len(set(rv.tolist())) == len(rv) and (a + i) not in rv.tolist()
        assert valid.sum(1).min() >= 1
    assert depth_seen == set(range(ix.n_depth))


def test_builder_deterministic(small_index, tmp_path):
    w, path = small_index
    p1 = str(tmp_path / "t1.esgi")
    esg.build_index(w["X"], w["attr"].astype(np.float64), p1, degree=12, leaf=100,
                    ef_construction=64, threads=1)
    assert open(p1, "rb").read() == open(path, "rb").read()


def test_builder_errors(tmp_path):
    X = np.zeros((10, 4), np.float32)
    with pytest.raises(esg.EsgError) as e:
        esg.build_index(X, np.arange(10.0), str(tmp_path / "x"), leaf=0)
    assert e.value.status == esg.ESG_EINVAL
    with pytest.raises(esg.EsgError) as e:
        esg.build_index(X, np.full(10, np.nan), str(tmp_path / "x"))
    assert e.value.status == esg.ESG_EINVAL
    with pytest.raises(esg.EsgError) as e:
        esg.build_index(X, np.arange(10.0), "/nonexistent_dir/x.esgi")
    assert e.value.status == esg.ESG_EIO


def _crc32c(data: bytes) -> int:
    """CRC-32C (Castagnoli, reflected polynomial 0x82F63B78), bit by bit."""
    crc = 0xFFFFFFFF
    for byte in data:
        crc ^= byte
        for _ in range(8):
            crc = (crc >> 1) ^ (0x82F63B78 if crc & 1 else 0)
    return crc ^ 0xFFFFFFFF


def test_crc32c_check_value():
    # the standard check value of CRC-32C over the ASCII digits 1..9
    assert _crc32c(b"123456789") == 0xE3069283


def _load_status(path):
    import ctypes
    h = ctypes.c_void_p()
    st = esg.lib().esg_load_index(path.encode(), 0, ctypes.byref(h))
    if st == 0:
        esg.lib().esg_free_index(h)
    return st


def test_loader_rejects_malformed(small_index, tmp_path):
    w, path = small_index
    raw = bytearray(open(path, "rb").read())
    assert _load_status(str(tmp_path / "missing.esgi")) == esg.ESG_EIO

    def variant(name, data):
        p = str(tmp_path / name)
        open(p, "wb").write(bytes(data))
        return _load_status(p)

    bad = raw.copy(); bad[0] ^= 1
    assert variant("magic", bad) == esg.ESG_EFORMAT
    assert variant("trunc", raw[:-100]) == esg.ESG_EFORMAT
    bad = raw.copy(); bad[-8] ^= 0x40                      # entry-point section byte
    assert variant("crc", bad) == esg.ESG_EFORMAT
    bad = raw.copy(); bad[20] ^= 1                          # header field (n)
    assert variant("hdr", bad) == esg.ESG_EFORMAT
    # c = 1 / c_den above 1 / fanout: Alg. 4 could select more than two parts
    # (Lemma 4.2 needs c <= 1/2); a consistent header (checksum rewritten)
    # with c_den = 1 must still be refused
    bad = raw.copy()
    assert struct.unpack_from("<i", bad, 44)[0] == 2        # c_den
    struct.pack_into("<i", bad, 44, 1)
    struct.pack_into("<I", bad, 124, _crc32c(bytes(bad[:124])))
    assert variant("cden", bad) == esg.ESG_EFORMAT
    # a well-formed file: loads where a device exists, reports the missing device here
    assert _load_status(path) in (esg.ESG_OK, esg.ESG_EHIP)
