"""The C-ABI library: it loads, exports every symbol include/ccfmm.h declares,
and rejects invalid arguments before touching a GPU.  CPU only."""
import os
import re

import numpy as np
import pytest

from paper_0810_0233_amd import ccfmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "ccfmm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ccfmm_[a-z0-9_]+)\s*\(", txt)))


def test_header_declarations_match_binding():
    assert declared_symbols() == sorted(ccfmm.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = ccfmm.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_status_strings_and_defaults():
    assert ccfmm.status_string(ccfmm.OK) == "ok"
    assert ccfmm.status_string(ccfmm.EINVAL) == "invalid argument"
    p = ccfmm.params()
    assert p.order == 4 and p.theta == 0.5 and p.max_batch == 1
    assert p.keep_lists == 1 and p.truncation == 0 and p.m2l_traceless == 1
    assert p.m2l_variant == -1  # chosen at plan creation


@pytest.mark.parametrize("bad", [dict(order=0), dict(order=9), dict(theta=0.0), dict(theta=1.0),
                                 dict(max_batch=0), dict(precision=7), dict(truncation=2),
                                 dict(m2l_traceless=3), dict(max_batch=4097), dict(leaf_rule=2),
                                 dict(selector=2), dict(selector=1, order=1), dict(selector=1, err_bound=0.0),
                                 dict(selector=1, sel_margin=-0.1), dict(leaf_target=float("inf")),
                                 dict(device_mem_cap=-1)])
def test_invalid_params_rejected_without_gpu(bad):
    prm = ccfmm.params(**bad)
    with pytest.raises(ccfmm.CCFMMError) as e:
        ccfmm.Plan.create(np.zeros((4, 3)), prm)
    assert e.value.status == ccfmm.EINVAL


def test_empty_input_rejected():
    # no dipoles: nothing to build a tree on; refused before any device call
    with pytest.raises(ccfmm.CCFMMError) as e:
        ccfmm.Plan.create(np.zeros((0, 3)), ccfmm.params())
    assert e.value.status == ccfmm.EINVAL
    assert "n must be >= 1" in ccfmm.last_error()


def test_nonfinite_positions_rejected():
    pos = np.zeros((4, 3))
    pos[2, 1] = np.nan
    with pytest.raises(ccfmm.CCFMMError) as e:
        ccfmm.Plan.create(pos, ccfmm.params())
    assert e.value.status == ccfmm.EINVAL
    assert "non-finite" in ccfmm.last_error()


def test_energy_helper_matches_definition():
    rng = np.random.default_rng(0)
    m = rng.normal(size=(2, 10, 3))
    H = rng.normal(size=(2, 10, 3))
    E = ccfmm.energy(m, H)
    np.testing.assert_allclose(E, -0.5 * np.sum(m * H, axis=(1, 2)), rtol=1e-14)


def test_noalloc_energy_rejects_sizes_without_gpu():
    # argument checks come before any device call
    for n, nb in ((0, 1), (10, 0), (10, ccfmm.NOALLOC_MAX_BATCH + 1)):
        with pytest.raises(ccfmm.CCFMMError) as e:
            ccfmm.energy_device_noalloc(n, nb, 8, 8, 8)
        assert e.value.status == ccfmm.EINVAL
    assert "nbatch must be in 1..%d" % ccfmm.NOALLOC_MAX_BATCH in ccfmm.last_error()


def fnv1a64(b):
    h = 14695981039346656037
    for x in b:
        h = ((h ^ x) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def test_selector_file_format_and_checks(tmp_path):
    """The weights file has the documented little-endian layout, reads back
    bit for bit, a missing file is a warning, and any altered, truncated or
    foreign file is refused."""
    import struct

    rng = np.random.default_rng(5)
    P = rng.standard_normal(ccfmm.MLP_PARAMS).astype(np.float32)
    f = tmp_path / "w.ccsel"
    ccfmm.selector_write(str(f), P)
    b = f.read_bytes()
    assert len(b) == 8 + 7 * 4 + 5 * 8 + 4 * ccfmm.MLP_PARAMS + 8
    assert b[:8] == b"CCFMMSEL"
    assert struct.unpack_from("<7I", b, 8) == (1, 8, 64, 25, ccfmm.MLP_PARAMS, 2, 6)
    assert struct.unpack_from("<5d", b, 36) == (0.3, 0.4, 0.5, 0.6, 0.7)
    assert np.array_equal(np.frombuffer(b, dtype="<f4", count=ccfmm.MLP_PARAMS, offset=76), P)
    assert struct.unpack_from("<Q", b, len(b) - 8)[0] == fnv1a64(b[:-8])
    assert np.array_equal(ccfmm.selector_read(str(f)), P)
    # missing file: warning, nothing read
    assert ccfmm.selector_read(str(tmp_path / "absent.ccsel")) is None
    assert ccfmm.lib().ccfmm_selector_read(str(tmp_path / "absent.ccsel").encode(), None) == ccfmm.W_NOWEIGHTS
    # one parameter bit flipped, truncated, foreign header: refused
    bad = bytearray(b)
    bad[100] ^= 1
    for name, data in (("flip", bytes(bad)), ("short", b[:-1]), ("magic", b"CCFMMSEX" + b[8:]),
                       ("version", b[:8] + struct.pack("<I", 2) + b[12:])):
        g = tmp_path / (name + ".ccsel")
        g.write_bytes(data)
        with pytest.raises(ccfmm.CCFMMError) as e:
            ccfmm.selector_read(str(g))
        assert e.value.status == ccfmm.EINVAL


def test_selector_train_rejects_bad_specs_without_gpu():
    pos = np.zeros((4, 3))
    g = [dict(pos=pos, m=pos, box=None)]
    for kw in (dict(order=1), dict(theta=1.0), dict(steps=0), dict(lr=0.0)):
        with pytest.raises(ccfmm.CCFMMError) as e:
            ccfmm.selector_train(g, **kw)
        assert e.value.status == ccfmm.EINVAL
    with pytest.raises(ccfmm.CCFMMError) as e:
        ccfmm.selector_train([])
    assert e.value.status == ccfmm.EINVAL


STRUCTS = ("ccfmm_params", "ccfmm_tune_entry", "ccfmm_info", "ccfmm_train_geometry", "ccfmm_train_spec",
           "ccfmm_train_info", "ccfmm_pass_times", "ccfmm_select_info")


def test_binding_struct_layouts_match_header(tmp_path):
    """Every struct of the binding has the size and field offsets the C
    compiler gives the header's struct (a C program built against
    include/ccfmm.h prints them)."""
    import ctypes
    import subprocess

    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "ccfmm.h"', "int main(void) {"]
    for sname in STRUCTS:
        S = getattr(ccfmm, sname)
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (sname, sname))
        for fname, _ in S._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (sname, fname, sname, fname))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {}
    for ln in out:
        if ln.strip():
            a, b, v = ln.split()
            got[(a, b)] = int(v)
    for sname in STRUCTS:
        S = getattr(ccfmm, sname)
        assert got[(sname, "size")] == ctypes.sizeof(S), sname
        for fname, _ in S._fields_:
            assert got[(sname, fname)] == getattr(S, fname).offset, (sname, fname)
