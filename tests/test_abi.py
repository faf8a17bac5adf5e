"""The C-ABI library: it loads, exports every function include/*.h
declares, and its host-only helpers (segmentation, table, QPP) agree with
the oracle.  No GPU needed."""
import ctypes as ct
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1905_01141_amd as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    inc = os.path.join(ROOT, "include")
    src = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc))
                  if f.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"^\s*#.*$", "", src, flags=re.M)  # preprocessor lines (macros are not symbols)
    names = re.findall(r"\b([A-Za-z_][A-Za-z0-9_]*)\s*\([^;{]*\)\s*;", src)
    return sorted(set(n for n in names if n not in ("sizeof",)))


def test_library_exports_every_declared_function():
    L = ct.CDLL(T.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(T.EXPORTS)


def test_host_helpers_agree_with_oracle(orc):
    assert np.array_equal(T.k_table(), orc.k_table())
    for K in T.k_table().tolist():
        pi, f1, f2 = T.qpp(K)
        assert (f1, f2) == orc.qpp_params(K)
        assert np.array_equal(pi, orc.qpp(K))
    rng = np.random.default_rng(1)
    for tbs in list(range(1, 300)) + rng.integers(1, 1 << 20, 200).tolist() + [6120, 6121]:
        assert T.segment(int(tbs)) == orc.segment(int(tbs))
        assert T.tb_llr_count(int(tbs)) == orc.tb_llr_count(int(tbs))
    with pytest.raises(T.TdecError):
        T.segment(0)
    with pytest.raises(T.TdecError):
        T.segment((1 << 20) + 1)


def test_binding_rejects_oversized_descriptors():
    """The binding refuses descriptors that would reach past a tensor."""
    import torch
    descs, n_llr, n_bytes = T.make_descs([(6144, 0, T.CRC24B)] * 2)
    small = torch.zeros(n_llr - 1, dtype=torch.int16)
    with pytest.raises(ValueError):
        T._need(small, "int16", n_llr, "llr")
    with pytest.raises(ValueError):
        T._need(torch.zeros(n_llr, dtype=torch.int32), "int16", n_llr, "llr")
    T._need(torch.zeros(n_llr, dtype=torch.int16), "int16", n_llr, "llr")


def test_segmentation_matches_oracle_for_every_size(orc):
    """The library's segmentation (closed-form K+) equals the oracle's for
    every transport block size 1..2^20."""
    L = T.lib()
    OL = orc.lib()
    s1 = T.Seg()

    class OSeg(ct.Structure):
        _fields_ = [(n, ct.c_int32) for n in ("B", "C", "L", "Kplus", "Kminus", "Cplus",
                                               "Cminus", "F")]
    s2 = OSeg()
    OL.or_segment.argtypes = [ct.c_int32, ct.c_void_p]
    bad = 0
    for tbs in range(1, (1 << 20) + 1):
        r1 = L.tdec_segment(tbs, ct.byref(s1))
        r2 = OL.or_segment(tbs, ct.byref(s2))
        if (r1 == 0) != (r2 == 0) or (r1 == 0 and bytes(s1) != bytes(s2)):
            bad += 1
    assert bad == 0


def test_c_example_builds_against_the_header_alone(tmp_path):
    """The C ABI is usable from plain C: the example compiles with gcc -std=c99
    -Werror against include/tdec.h and links against libtdec.so."""
    from paper_1905_01141_amd import build as B
    out = str(tmp_path / "tb_roundtrip")
    r = subprocess.run(B.example_cmd(out), capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert os.path.exists(out)


def test_probes_check_their_arguments():
    """The device probes refuse bad arguments before touching a device."""
    L = T.lib()
    d = ct.c_double()
    assert L.tdec_probe_valu_int16(0, 0, ct.byref(d)) == -1
    assert L.tdec_probe_valu_int16(0, 1000001, ct.byref(d)) == -1
    assert L.tdec_probe_valu_int16(0, 10, None) == -1
    assert L.tdec_probe_hbm(0, 1 << 20, ct.byref(d), ct.byref(d)) == -1      # below 16 MiB
    assert L.tdec_probe_hbm(0, (16 << 20) + 8, ct.byref(d), ct.byref(d)) == -1  # not a multiple of 16
    assert L.tdec_probe_launch(0, 0, ct.byref(d), ct.byref(d)) == -1
