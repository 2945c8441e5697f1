"""C-ABI checks that need no GPU: the library loads, exports every function that
include/qfs.h declares, the binding's struct layouts match the header (checked by
compiling a probe against the header with gcc), defaults are App. A's recommended
hyperparameters, and argument validation rejects bad input before any device work."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2405_12866_amd import qfs as Q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qfs.h")


def _declared():
    src = open(HEADER).read()
    return re.findall(r"^(?:int|void|const char \*)\s*\*?\s*(qfs_\w+)\s*\(", src, re.M)


def test_library_exports_every_declared_function():
    lib = Q.load()
    names = _declared()
    assert len(names) >= 14
    assert sorted(names) == sorted(Q.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n
    assert lib.qfs_version().decode().startswith("qfs-hip")


def test_struct_layouts_match_header(tmp_path):
    probe = tmp_path / "probe.c"
    probe.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "qfs.h"\n'
        "int main(void){\n"
        ' printf("%zu %zu %zu %zu %zu\\n", sizeof(qfs_template), sizeof(qfs_target),'
        " sizeof(qfs_params), sizeof(qfs_result), sizeof(qfs_c128));\n"
        ' printf("%zu %zu %zu\\n", offsetof(qfs_params, hip_stream),'
        " offsetof(qfs_result, sweep_seconds), offsetof(qfs_target, n_val));\n"
        " return 0;}\n")
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(probe), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    got = [int(x) for x in out]
    want = [C.sizeof(Q.Template), C.sizeof(Q.Target), C.sizeof(Q.Params), C.sizeof(Q.Result), 16,
            Q.Params.hip_stream.offset, Q.Result.sweep_seconds.offset, Q.Target.n_val.offset]
    assert got == want


def test_default_params_are_paper_recommendations():
    p = Q.qfs_default_params()
    assert p["dist_tol"] == 1e-8 and p["diff_tol_r"] == 1e-5 and p["plateau_window"] == 5
    assert p["min_iter"] == 6 and p["max_iter"] == 10000 and p["m_init"] == 2
    assert p["overtrain_ratio"] == 0.1 and p["multistarts"] == 16 and p["beta"] == 0.0
    assert p["precision"] == Q.QFS_PREC_MIXED and p["refine_below"] == 1e-5


def test_strerror_covers_codes():
    lib = Q.load()
    texts = {c: lib.qfs_strerror(c).decode() for c in range(6)}
    assert texts[0] == "ok" and len(set(texts.values())) == 6


@pytest.mark.parametrize("pairs,n", [([(0, 0)], 3), ([(0, 3)], 3), ([(-1, 1)], 3), ([(0, 1)], 1),
                                     ([(0, 1)], 25)])
def test_invalid_templates_rejected_without_device_work(pairs, n):
    lib = Q.load()
    arr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32))
    pp = arr.ctypes.data_as(C.POINTER(C.c_int32))
    c = np.zeros(1)
    rc = lib.qfs_sweep(n, 1, pp, None, 1, C.c_void_p(16), C.c_void_p(16), 1, C.c_void_p(16), 0,
                       0.0, 0, c.ctypes.data_as(C.c_void_p), None)
    assert rc == Q.QFS_EINVAL
    tmpl = Q.Template(n, 1, pp)
    par = Q.Params()
    lib.qfs_default_params(C.byref(par))
    res = Q.Result()
    tgt = Q.Target()
    rc = lib.qfs_instantiate(C.byref(tmpl), C.byref(tgt), C.byref(par), None, C.c_void_p(16),
                             C.byref(res))
    assert rc == Q.QFS_EINVAL
    assert "template" in lib.qfs_last_error_detail().decode()


@pytest.mark.parametrize("kinds,fixed", [([0, 3], None), ([0, -1], None), ([1, 2], None)])
def test_invalid_gate_kinds_rejected_without_device_work(kinds, fixed):
    """An unknown kind, or a constant gate without fixed_gates, is QFS_EINVAL."""
    lib = Q.load()
    arr = np.ascontiguousarray(np.asarray([(0, 1), (1, 2)], dtype=np.int32))
    kd = np.ascontiguousarray(np.asarray(kinds, dtype=np.int32))
    tmpl = Q.Template(3, 2, arr.ctypes.data_as(C.POINTER(C.c_int32)),
                      kd.ctypes.data_as(C.POINTER(C.c_int32)), fixed)
    par = Q.Params()
    lib.qfs_default_params(C.byref(par))
    tgt = Q.Target()
    tgt.kind = Q.QFS_TARGET_DENSE
    tgt.U = C.c_void_p(16)
    res = Q.Result()
    rc = lib.qfs_instantiate(C.byref(tmpl), C.byref(tgt), C.byref(par), None, C.c_void_p(16),
                             C.byref(res))
    assert rc == Q.QFS_EINVAL
    assert "template" in lib.qfs_last_error_detail().decode()


def test_gate_kinds_unsupported_in_learned_entries():
    """The sample-count network takes two-qubit templates only; the batched engine checks
    the kinds before any device work."""
    lib = Q.load()
    arr = np.ascontiguousarray(np.asarray([(0, 1), (1, 2)], dtype=np.int32))
    kd = np.ascontiguousarray(np.asarray([1, 0], dtype=np.int32))
    tmpl = Q.Template(3, 2, arr.ctypes.data_as(C.POINTER(C.c_int32)),
                      kd.ctypes.data_as(C.POINTER(C.c_int32)), None)
    par = Q.Params()
    lib.qfs_default_params(C.byref(par))
    tgt = Q.Target()
    tgt.kind = Q.QFS_TARGET_DENSE
    tgt.U = C.c_void_p(16)
    res = Q.Result()
    out = (C.c_void_p * 1)(16)
    bad = np.ascontiguousarray(np.asarray([1, 5], dtype=np.int32))
    tmpl_bad = Q.Template(3, 2, arr.ctypes.data_as(C.POINTER(C.c_int32)),
                          bad.ctypes.data_as(C.POINTER(C.c_int32)), None)
    assert lib.qfs_instantiate_batch(1, C.byref(tmpl_bad), C.byref(tgt), C.byref(par), out,
                                     C.byref(res)) == Q.QFS_EINVAL
    f = np.zeros(64, dtype=np.float32)
    assert lib.qfs_features(C.byref(tmpl), f.ctypes.data_as(C.c_void_p)) == Q.QFS_EUNSUPPORTED


def test_invalid_params_rejected():
    lib = Q.load()
    arr = np.ascontiguousarray(np.asarray([(0, 1)], dtype=np.int32))
    tmpl = Q.Template(3, 1, arr.ctypes.data_as(C.POINTER(C.c_int32)))
    tgt = Q.Target()
    tgt.kind = Q.QFS_TARGET_DENSE
    tgt.U = C.c_void_p(16)
    for field, bad in [("multistarts", 0), ("m_init", 9), ("beta", 1.5), ("precision", 7),
                       ("max_iter", 0)]:
        par = Q.Params()
        lib.qfs_default_params(C.byref(par))
        setattr(par, field, bad)
        res = Q.Result()
        rc = lib.qfs_instantiate(C.byref(tmpl), C.byref(tgt), C.byref(par), None, C.c_void_p(16),
                                 C.byref(res))
        assert rc == Q.QFS_EINVAL, field


def test_qudit_target_arguments_rejected_without_device_work():
    """qfs_qudit_instantiate_target checks d, the template, the target and the params on
    the host before any device call."""
    lib = Q.load()
    arr = np.ascontiguousarray(np.asarray([(0, 1), (1, 2)], dtype=np.int32))
    tmpl = Q.Template(3, 2, arr.ctypes.data_as(C.POINTER(C.c_int32)))
    other = Q.Template(4, 2, arr.ctypes.data_as(C.POINTER(C.c_int32)))
    bad_pairs = np.ascontiguousarray(np.asarray([(0, 3)], dtype=np.int32))
    bad_circ = Q.Template(3, 1, bad_pairs.ctypes.data_as(C.POINTER(C.c_int32)))
    par = Q.Params()
    lib.qfs_default_params(C.byref(par))
    res = Q.Result()
    out = C.c_void_p(16)

    def call(d, tmpl_, tgt, p=par):
        return lib.qfs_qudit_instantiate_target(d, C.byref(tmpl_), C.byref(tgt), C.byref(p), None, out,
                                                C.byref(res))

    dense = Q.Target()
    dense.kind = Q.QFS_TARGET_DENSE
    dense.U = C.c_void_p(16)
    assert call(5, tmpl, dense) == Q.QFS_EUNSUPPORTED
    assert call(1, tmpl, dense) == Q.QFS_EUNSUPPORTED
    no_u = Q.Target()
    no_u.kind = Q.QFS_TARGET_DENSE
    assert call(3, tmpl, no_u) == Q.QFS_EINVAL
    big = Q.Template(9, 2, arr.ctypes.data_as(C.POINTER(C.c_int32)))  # 4^9 > 2^16 amplitudes
    assert call(4, big, dense) == Q.QFS_EINVAL
    for ct in (other, bad_circ):
        circ = Q.Target()
        circ.kind = Q.QFS_TARGET_CIRCUIT
        circ.circuit = C.pointer(ct)
        circ.circuit_gates = C.c_void_p(16)
        assert call(3, tmpl, circ) == Q.QFS_EINVAL
    unknown = Q.Target()
    unknown.kind = 7
    assert call(3, tmpl, unknown) == Q.QFS_EINVAL
    bad_kinds = np.ascontiguousarray(np.asarray([0, 7], dtype=np.int32))
    tmpl_k = Q.Template(3, 2, arr.ctypes.data_as(C.POINTER(C.c_int32)),
                        bad_kinds.ctypes.data_as(C.POINTER(C.c_int32)))
    assert call(3, tmpl_k, dense) == Q.QFS_EINVAL
    for field, bad in [("multistarts", 0), ("beta", 1.5), ("precision", 7), ("max_iter", 0),
                       ("full_unitary", 1)]:
        p = Q.Params()
        lib.qfs_default_params(C.byref(p))
        setattr(p, field, bad)
        assert call(3, tmpl, dense, p) == Q.QFS_EINVAL, field


def test_qudit_batch_arguments_rejected_without_device_work():
    lib = Q.load()
    par = Q.Params()
    lib.qfs_default_params(C.byref(par))
    tm = (Q.Template * 1)()
    tg = (Q.Target * 1)()
    ptrs = (C.c_void_p * 1)(None)
    res = (Q.Result * 1)()
    assert lib.qfs_qudit_instantiate_batch(3, 0, tm, tg, C.byref(par), ptrs, res) == Q.QFS_EINVAL
    assert lib.qfs_qudit_instantiate_batch(3, 1, None, tg, C.byref(par), ptrs, res) == Q.QFS_EINVAL
    assert lib.qfs_qudit_instantiate_batch(3, 1, tm, tg, None, ptrs, res) == Q.QFS_EINVAL
