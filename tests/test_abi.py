"""The C-ABI library loads and exports every symbol include/pch.h declares.

No compute calls: mesh validation errors are reported before any device work,
so they are checked here without a GPU.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "pch.h")).read()
    return sorted(set(re.findall(r"^\s*(?:pch_status|void|const char\*)\s+(pch_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def pch():
    from paper_1305_1293_amd import pch as P
    P.lib()
    return P


def test_every_declared_symbol_is_exported(pch):
    syms = declared_symbols()
    assert len(syms) >= 10
    L = ctypes.CDLL(pch.LIB_PATH)
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(pch.EXPORTS) == syms


def test_status_strings_and_defaults(pch):
    L = pch.lib()
    assert L.pch_status_string(0) == b"ok"
    assert L.pch_status_string(-2) == b"invalid mesh"
    o = pch.Options()
    L.pch_options_default(ctypes.byref(o))
    assert o.k == 16384 and o.filters == 3 and o.select_mode == 0 and o.eps_tiny == 0.0


def _code(pch, faces, xyz=None, he_len=None, nv=None):
    with pytest.raises(pch.PchError) as e:
        pch.Mesh(np.asarray(faces), xyz=None if xyz is None else np.asarray(xyz, float), he_len=he_len,
                 nv=nv, stream=0)
    return e.value.code


def test_invalid_meshes_rejected_before_device_work(pch):
    xyz = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]]
    assert _code(pch, [[0, 1, 2], [1, 0, 3], [0, 1, 4]], xyz) == -2       # edge with three faces
    assert _code(pch, [[0, 1, 2], [0, 1, 3]], xyz) == -2                   # flipped neighbour
    assert _code(pch, [[0, 1, 2]], [[0, 0, 0], [1, 0, 0], [2, 0, 0]]) == -2  # zero area
    assert _code(pch, [[0, 1, 9]], xyz) == -1                              # index out of range
    bow = [[0, 0, 0], [1, 0, 0], [1, 1, 0], [-1, 0, 0], [-1, -1, 0]]
    assert _code(pch, [[0, 1, 2], [0, 3, 4]], bow) == -2                   # two fans at a vertex
    assert _code(pch, [[0, 1, 2]], he_len=np.array([1.0, 1.0, 3.0]), nv=3) == -2  # lengths violate triangle ineq.
    assert _code(pch, [[0, 1, 2]], he_len=np.array([1.0, -1.0, 1.0]), nv=3) == -1


def test_field_status_codes_match_header(pch):
    text = open(os.path.join(ROOT, "include", "pch.h")).read()
    codes = {name: int(v) for name, v in re.findall(r"(PCH_FIELD_\w+)\s*=\s*(\d+)", text)}
    assert codes == {v: k for k, v in pch.FIELD_STATUS.items()}
    names = {c: pch.field_status_string(c) for c in pch.FIELD_STATUS}
    assert names[0] == "ok"
    assert len(set(names.values())) == len(names)  # every status has its own message
    assert "non-finite" in names[5] and "outside the mesh" in names[6]
    assert all("rerun" in names[c] for c in (1, 2, 3, 4))  # the statuses a rerun completes
    assert pch.field_status_string(99) == "unknown field status"


def test_tune_cache_round_trip(pch, tmp_path):
    src = tmp_path / "in.txt"
    src.write_text("# comment\ngfx950 20 29 9 32768 512 1 4 8 213.800\ngfx950 17 25 6 8192 256 1 1 2 12.500\n")
    pch.tune_cache_load(str(src))
    out = tmp_path / "out.txt"
    pch.tune_cache_save(str(out))
    lines = [l for l in out.read_text().splitlines() if not l.startswith("#")]
    assert "gfx950 20 29 9 32768 512 1 4 8 213.800" in lines
    assert "gfx950 17 25 6 8192 256 1 1 2 12.500" in lines
    bad = tmp_path / "bad.txt"
    bad.write_text("gfx950 20 29 9 32768 300 1 4 8 1.0\n")  # no such workgroup size
    with pytest.raises(pch.PchError) as e:
        pch.tune_cache_load(str(bad))
    assert e.value.code == -1
    with pytest.raises(pch.PchError):
        pch.tune_cache_load(str(tmp_path / "missing.txt"))
