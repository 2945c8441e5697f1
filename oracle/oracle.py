"""ctypes wrapper of the C oracle (test infrastructure only; see package docstring).

Arrays are numpy complex128, sample-major ``[M][N]``; gates are ``[L][4][4]``
row-major ``u[q][p]`` with local index ``2*bit(qa) + bit(qb)`` and qubit 0 the most
significant bit of the amplitude index.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qfs_oracle.c")
_LIB = os.path.join(_HERE, "libqfs_oracle.so")
_lock = threading.Lock()
_lib = None

ROLE_TRAIN, ROLE_VAL, ROLE_INIT = 1, 2, 3
TARGET_DENSE, TARGET_CIRCUIT, TARGET_SAMPLES = 0, 1, 2
GATE_2Q, GATE_1Q, GATE_FIXED = 0, 1, 2
REASONS = {0: "SUCCESS", 1: "PLATEAU", 2: "MAX_ITER", 3: "NOT_GENERALIZED", 4: "TIMEOUT"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE arithmetic, OpenMP over starts)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-Wall",
               "-Wno-unused-function", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _C2(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class Params(C.Structure):
    _fields_ = [
        ("dist_tol", C.c_double),
        ("diff_tol_r", C.c_double),
        ("plateau_window", C.c_int32),
        ("min_iter", C.c_int32),
        ("max_iter", C.c_int64),
        ("m_init", C.c_int32),
        ("m_max", C.c_int32),
        ("overtrain_ratio", C.c_double),
        ("multistarts", C.c_int32),
        ("beta", C.c_double),
        ("seed", C.c_uint64),
        ("fixed_m", C.c_int32),
        ("m_val", C.c_int32),
        ("beta_normalized", C.c_int32),
    ]


class Result(C.Structure):
    _fields_ = [
        ("reason", C.c_int32),
        ("m_final", C.c_int32),
        ("sweeps", C.c_int32),
        ("restarts", C.c_int32),
        ("best_start", C.c_int32),
        ("m_total", C.c_int32),
        ("c_train", C.c_double),
        ("c_val", C.c_double),
        ("seconds", C.c_double),
    ]


class Trace(C.Structure):
    _fields_ = [
        ("capacity", C.c_int32),
        ("count", C.c_int32),
        ("start", C.POINTER(C.c_int32)),
        ("sweep", C.POINTER(C.c_int32)),
        ("m", C.POINTER(C.c_int32)),
        ("c_train", C.POINTER(C.c_double)),
        ("c_val", C.POINTER(C.c_double)),
        ("iter", C.POINTER(C.c_int32)),
        ("event", C.POINTER(C.c_int32)),
        ("dbl_capacity", C.c_int32),
        ("dbl_count", C.c_int32),
        ("dbl_rows", C.c_int32),
        ("dbl_m_old", C.POINTER(C.c_int32)),
        ("dbl_m_new", C.POINTER(C.c_int32)),
        ("dbl_gates_before", C.c_void_p),
        ("dbl_gates_after", C.c_void_p),
        ("dbl_psi", C.c_void_p),
        ("dbl_phi", C.c_void_p),
        ("dbl_c_prev", C.POINTER(C.c_double)),
    ]


# control decision recorded per trace row (trace["event"])
EV_RUN, EV_SUCCESS, EV_OVERTRAINED, EV_NOT_GEN, EV_PLATEAU, EV_MAX_ITER = range(6)


def default_params(**kw) -> dict:
    """App. A recommended hyperparameters (dist_tol 1e-8, window 5, diff_tol_r 1e-5,
    M0 2, overtrain_ratio 0.1, min_iter 6, max_iter 1e4, 16 multistarts, beta 0)."""
    p = dict(dist_tol=1e-8, diff_tol_r=1e-5, plateau_window=5, min_iter=6, max_iter=10000,
             m_init=2, m_max=0, overtrain_ratio=0.1, multistarts=16, beta=0.0, seed=0,
             fixed_m=0, m_val=0, beta_normalized=0)
    p.update(kw)
    return p


def load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.qo_philox4x32_10.argtypes = [P, P, P]
        lib.qo_cgauss.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64]
        lib.qo_cgauss.restype = _C2
        lib.qo_ginibre.argtypes = [C.c_int64, C.c_int64, C.c_uint64, C.c_uint32, C.c_uint32, P]
        lib.qo_orthonormalize.argtypes = [C.c_int64, C.c_int64, P]
        lib.qo_orthonormalize.restype = C.c_int
        lib.qo_draw_states.argtypes = [C.c_int, C.c_int, C.c_uint64, C.c_uint32, C.c_uint32, P]
        lib.qo_draw_states.restype = C.c_int
        lib.qo_haar_gate.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, P]
        lib.qo_haar_gate2.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, P]
        lib.qo_initial_gate.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_int, P, P]
        lib.qo_apply_gate.argtypes = [C.c_int, C.c_int, P, C.c_int, C.c_int, P]
        lib.qo_apply_gate_dag.argtypes = [C.c_int, C.c_int, P, C.c_int, C.c_int, P]
        lib.qo_apply_circuit.argtypes = [C.c_int, C.c_int, P, C.c_int, P, P]
        lib.qo_dense_apply.argtypes = [C.c_int, C.c_int, P, P, P]
        lib.qo_environment.argtypes = [C.c_int, C.c_int, P, P, C.c_int, C.c_int, P]
        lib.qo_environment1.argtypes = [C.c_int, C.c_int, P, P, C.c_int, P]
        lib.qo_svd4.argtypes = [P, P, P, P]
        lib.qo_update_gate.argtypes = [P, C.c_double, P]
        lib.qo_update_gate1.argtypes = [P, C.c_double, P]
        lib.qo_state_distance.argtypes = [C.c_int, C.c_int, P, P]
        lib.qo_state_distance.restype = C.c_double
        lib.qo_sweep.argtypes = [C.c_int, C.c_int, P, P, C.c_int, P, P, P, C.c_double, C.c_double,
                                 P, P, P]
        lib.qo_sweep.restype = C.c_double
        lib.qo_instantiate.argtypes = [C.c_int, C.c_int, P, P, P, C.c_int, P, C.c_int, P, P, P, P,
                                       C.c_int, C.c_int, C.POINTER(Params), P, P,
                                       C.POINTER(Result), C.POINTER(Trace)]
        lib.qo_instantiate.restype = C.c_int
        lib.qd_apply_gate.argtypes = [C.c_int, C.c_int, C.c_int, P, C.c_int, C.c_int, P, C.c_int]
        lib.qd_environment.argtypes = [C.c_int, C.c_int, C.c_int, P, P, C.c_int, C.c_int, P]
        lib.qd_svd.argtypes = [C.c_int, P, P, P, P]
        lib.qd_update_gate.argtypes = [C.c_int, P, C.c_double, P]
        lib.qd_haar_gate.argtypes = [C.c_int, C.c_uint64, C.c_uint32, C.c_uint32, P]
        lib.qd_sweep.argtypes = [C.c_int, C.c_int, C.c_int, P, P, C.c_int, P, P, P, C.c_double,
                                 C.c_double, P, P]
        lib.qd_sweep.restype = C.c_double
        lib.qd_instantiate.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, P, P, C.c_int, C.c_int,
                                       C.POINTER(Params), P, P, C.POINTER(Result), C.POINTER(Trace)]
        lib.qd_instantiate.restype = C.c_int
        lib.qd_draw_states.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_uint32, C.c_uint32,
                                       P]
        lib.qd_draw_states.restype = C.c_int
        lib.qd_environment1.argtypes = [C.c_int, C.c_int, C.c_int, P, P, C.c_int, P]
        lib.qd_update_gate1.argtypes = [C.c_int, P, C.c_double, P]
        lib.qd_haar_gate1.argtypes = [C.c_int, C.c_uint64, C.c_uint32, C.c_uint32, P]
        lib.qd_instantiate_target.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, C.c_int, P, C.c_int, P, P,
                                              C.POINTER(Params), P, P, C.POINTER(Result),
                                              C.POINTER(Trace)]
        lib.qd_instantiate_target.restype = C.c_int
        _lib = lib
        return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _pairs(pairs):
    return np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    load().qo_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def cgauss(seed, role, stream, idx):
    r = load().qo_cgauss(seed, role, stream, idx)
    return complex(r.re, r.im)


def ginibre(rows, cols, seed, role, stream):
    out = np.zeros((cols, rows), dtype=np.complex128)
    load().qo_ginibre(rows, cols, seed, role, stream, _p(out))
    return out


def orthonormalize(cols_major):
    a = _c128(cols_major).copy()
    rc = load().qo_orthonormalize(a.shape[1], a.shape[0], _p(a))
    if rc != 0:
        raise ValueError("dependent columns")
    return a


def draw_states(n, M, seed, role=ROLE_TRAIN, stream=0):
    out = np.zeros((M, 1 << n), dtype=np.complex128)
    rc = load().qo_draw_states(n, M, seed, role, stream, _p(out))
    if rc != 0:
        raise ValueError("dependent columns")
    return out


def haar_gate(seed, start, gate):
    u = np.zeros((4, 4), dtype=np.complex128)
    load().qo_haar_gate(seed, start, gate, _p(u))
    return u


def haar_gate2(seed, start, gate):
    v = np.zeros((2, 2), dtype=np.complex128)
    load().qo_haar_gate2(seed, start, gate, _p(v))
    return v


def _kinds(kinds, L):
    if kinds is None:
        return None
    k = np.ascontiguousarray(np.asarray(kinds, dtype=np.int32).reshape(-1))
    if k.shape[0] != L:
        raise ValueError("kinds needs one entry per gate")
    return k


def initial_gates(seed, start, kinds, fixed=None):
    """Initial [L][4][4] slots of one start by gate kind."""
    k = _kinds(kinds, len(kinds))
    fx = None if fixed is None else _c128(fixed)
    out = np.zeros((k.shape[0], 4, 4), dtype=np.complex128)
    for i in range(k.shape[0]):
        load().qo_initial_gate(seed, start, i, int(k[i]), _p(fx), _p(out[i]))
    return out


def kron_i2(v):
    """The 4x4 slot of a one-qubit gate v: v (x) I_2."""
    return np.kron(np.asarray(v, dtype=np.complex128), np.eye(2))


def apply_gate(n, states, qa, qb, u, dagger=False):
    st = _c128(states).copy()
    M = st.shape[0]
    uu = _c128(u)
    f = load().qo_apply_gate_dag if dagger else load().qo_apply_gate
    f(n, M, _p(st), qa, qb, _p(uu))
    return st


def apply_circuit(n, states, pairs, gates):
    st = _c128(states).copy()
    pr = _pairs(pairs)
    g = _c128(gates)
    load().qo_apply_circuit(n, st.shape[0], _p(st), pr.shape[0], _p(pr), _p(g))
    return st


def dense_apply(n, U, states):
    st = _c128(states)
    out = np.zeros_like(st)
    load().qo_dense_apply(n, st.shape[0], _p(_c128(U)), _p(st), _p(out))
    return out


def environment(n, a, b, qa, qb):
    aa, bb = _c128(a), _c128(b)
    G = np.zeros((4, 4), dtype=np.complex128)
    load().qo_environment(n, aa.shape[0], _p(aa), _p(bb), qa, qb, _p(G))
    return G


def environment1(n, a, b, qa):
    aa, bb = _c128(a), _c128(b)
    G = np.zeros((2, 2), dtype=np.complex128)
    load().qo_environment1(n, aa.shape[0], _p(aa), _p(bb), qa, _p(G))
    return G


def update_gate1(G, beta=0.0, u=None):
    """One-qubit update; u is the 4x4 slot v (x) I_2 (read when beta != 0)."""
    uu = np.zeros((4, 4), dtype=np.complex128) if u is None else _c128(u).copy()
    load().qo_update_gate1(_p(_c128(G)), beta, _p(uu))
    return uu


def svd4(G):
    g = _c128(G)
    W = np.zeros((4, 4), dtype=np.complex128)
    V = np.zeros((4, 4), dtype=np.complex128)
    s = np.zeros(4)
    load().qo_svd4(_p(g), _p(W), _p(s), _p(V))
    return W, s, V


def update_gate(G, beta=0.0, u=None):
    uu = np.zeros((4, 4), dtype=np.complex128) if u is None else _c128(u).copy()
    load().qo_update_gate(_p(_c128(G)), beta, _p(uu))
    return uu


def state_distance(n, x, y):
    xx, yy = _c128(x), _c128(y)
    return load().qo_state_distance(n, xx.shape[0], _p(xx), _p(yy))


def sweep(n, pairs, psi, phi, gates, beta=0.0, record=False, kinds=None, gamma_scale=1.0):
    """One sweep; returns (new_gates, c_train) or, with record, also f_before, f_after
    and the environments. kinds: per-gate GATE_2Q / GATE_1Q / GATE_FIXED (None: all 2Q).
    gamma_scale multiplies each environment before the beta mix (1/M: normalised)."""
    pr = _pairs(pairs)
    L = pr.shape[0]
    kd = _kinds(kinds, L)
    g = _c128(gates).copy()
    ps, ph = _c128(psi), _c128(phi)
    fb = np.zeros(L) if record else None
    fa = np.zeros(L) if record else None
    gam = np.zeros((L, 4, 4), dtype=np.complex128) if record else None
    c = load().qo_sweep(n, L, _p(pr), _p(kd), ps.shape[0], _p(ps), _p(ph), _p(g), beta,
                        gamma_scale, _p(fb),
                        _p(fa), _p(gam))
    if record:
        return g, c, fb, fa, gam
    return g, c


def _int_ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _dbl_ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _make_trace(capacity, dbl_capacity, starts, L, gate_entries, n_amp):
    """Trace buffers (numpy) and the ctypes struct pointing at them. Doubling records
    hold every start's gates before/after, the training set (up to n_amp rows of n_amp
    amplitudes) and the plateau reference of each start on the new set."""
    bufs = dict(start=np.zeros(capacity, np.int32), sweep=np.zeros(capacity, np.int32),
                m=np.zeros(capacity, np.int32), c_train=np.zeros(capacity),
                c_val=np.zeros(capacity), iter=np.zeros(capacity, np.int32),
                event=np.full(capacity, -1, np.int32))
    dcap = max(int(dbl_capacity), 0)
    dbl = dict(m_old=np.zeros(max(dcap, 1), np.int32), m_new=np.zeros(max(dcap, 1), np.int32),
               gates_before=np.zeros((max(dcap, 1), starts, L, gate_entries), np.complex128),
               gates_after=np.zeros((max(dcap, 1), starts, L, gate_entries), np.complex128),
               psi=np.zeros((max(dcap, 1), n_amp, n_amp), np.complex128),
               phi=np.zeros((max(dcap, 1), n_amp, n_amp), np.complex128),
               c_prev=np.zeros((max(dcap, 1), starts)))
    tr = Trace(capacity, 0, _int_ptr(bufs["start"]), _int_ptr(bufs["sweep"]), _int_ptr(bufs["m"]),
               _dbl_ptr(bufs["c_train"]), _dbl_ptr(bufs["c_val"]), _int_ptr(bufs["iter"]),
               _int_ptr(bufs["event"]), dcap, 0, n_amp, _int_ptr(dbl["m_old"]),
               _int_ptr(dbl["m_new"]), dbl["gates_before"].ctypes.data,
               dbl["gates_after"].ctypes.data, dbl["psi"].ctypes.data, dbl["phi"].ctypes.data,
               _dbl_ptr(dbl["c_prev"]))
    return tr, bufs, dbl


def _read_trace(tr, bufs, dbl):
    out = {key: v[:tr.count].copy() for key, v in bufs.items()}
    k = tr.dbl_count
    out["doublings"] = [
        dict(m_old=int(dbl["m_old"][i]), m_new=int(dbl["m_new"][i]),
             gates_before=dbl["gates_before"][i].copy(), gates_after=dbl["gates_after"][i].copy(),
             psi=dbl["psi"][i, :dbl["m_new"][i]].copy(), phi=dbl["phi"][i, :dbl["m_new"][i]].copy(),
             c_prev=dbl["c_prev"][i].copy())
        for i in range(k)]
    return out


def instantiate(n, pairs, *, U=None, target_pairs=None, target_gates=None, psi=None,
                phi=None, n_val=0, params=None, gates_in=None, trace_capacity=0, kinds=None,
                fixed=None, doubling_capacity=0):
    """Full QFactor-Sample instantiation. Exactly one target form: dense ``U``, a target
    circuit (``target_pairs`` + ``target_gates``), or fixed samples ``psi``/``phi``
    whose last ``n_val`` rows are the validation set. ``kinds`` and ``fixed`` ([L][4][4],
    read for fixed gates) describe a template with one-qubit and constant gates.
    With ``trace_capacity`` the result holds a per-sweep trace (costs, sweep index since
    the last restart, control decision) and, with ``doubling_capacity``, a record of each
    doubling (gates of every start before and after it, the new training set, the
    plateau reference on it). Returns (gates, result dict)."""
    lib = load()
    pr = _pairs(pairs)
    L = pr.shape[0]
    kd = _kinds(kinds, L)
    fx = None if fixed is None else _c128(fixed)
    par = Params(**(params or default_params()))
    keep = []
    if U is not None:
        kind = TARGET_DENSE
        Uc = _c128(U)
        keep.append(Uc)
        args = (_p(Uc), 0, None, None, None, None, 0, 0)
    elif target_pairs is not None:
        kind = TARGET_CIRCUIT
        tp = _pairs(target_pairs)
        tg = _c128(target_gates)
        keep += [tp, tg]
        args = (None, tp.shape[0], _p(tp), _p(tg), None, None, 0, 0)
    else:
        kind = TARGET_SAMPLES
        ps, ph = _c128(psi), _c128(phi)
        keep += [ps, ph]
        args = (None, 0, None, None, _p(ps), _p(ph), ps.shape[0], n_val)
    gi = None
    if gates_in is not None:
        gi = _c128(gates_in)
        keep.append(gi)
    out = np.zeros((L, 4, 4), dtype=np.complex128)
    res = Result()
    tr = None
    if trace_capacity or doubling_capacity:
        tr, bufs, dbl = _make_trace(max(trace_capacity, 1), doubling_capacity, par.multistarts
                                    if par.multistarts > 0 else 1, L, 16, 1 << n)
    rc = lib.qo_instantiate(n, L, _p(pr), _p(kd), _p(fx), kind, *args, C.byref(par), _p(gi), _p(out),
                            C.byref(res), C.byref(tr) if tr is not None else None)
    if rc != 0:
        raise ValueError(f"qo_instantiate failed: {rc}")
    info = {f: getattr(res, f) for f, _ in Result._fields_}
    info["reason_name"] = REASONS[res.reason]
    if tr is not None:
        info["trace"] = _read_trace(tr, bufs, dbl)
    return out, info


# ------------------------------------------------------------------------ qudits
def qd_apply_gate(d, n, states, qa, qb, u, dagger=False):
    st = _c128(states).copy()
    load().qd_apply_gate(d, n, st.shape[0], _p(st), qa, qb, _p(_c128(u)), 1 if dagger else 0)
    return st


def qd_apply_circuit(d, n, states, pairs, gates):
    st = _c128(states).copy()
    for (a, b), u in zip(_pairs(pairs), _c128(gates)):
        load().qd_apply_gate(d, n, st.shape[0], _p(st), int(a), int(b), _p(_c128(u)), 0)
    return st


def qd_environment(d, n, a, b, qa, qb):
    aa, bb = _c128(a), _c128(b)
    G = np.zeros((d * d, d * d), dtype=np.complex128)
    load().qd_environment(d, n, aa.shape[0], _p(aa), _p(bb), qa, qb, _p(G))
    return G


def qd_svd(G):
    g = _c128(G)
    D = g.shape[0]
    W = np.zeros((D, D), dtype=np.complex128)
    V = np.zeros((D, D), dtype=np.complex128)
    s = np.zeros(D)
    load().qd_svd(D, _p(g), _p(W), _p(s), _p(V))
    return W, s, V


def qd_update_gate(G, beta=0.0, u=None):
    g = _c128(G)
    D = g.shape[0]
    uu = np.zeros((D, D), dtype=np.complex128) if u is None else _c128(u).copy()
    load().qd_update_gate(D, _p(g), beta, _p(uu))
    return uu


def qd_haar_gate(d, seed, start, gate):
    u = np.zeros((d * d, d * d), dtype=np.complex128)
    load().qd_haar_gate(d, seed, start, gate, _p(u))
    return u


def qd_sweep(d, n, pairs, psi, phi, gates, beta=0.0, gamma_scale=1.0, record=False, kinds=None):
    pr = _pairs(pairs)
    L = pr.shape[0]
    kd = _kinds(kinds, L)
    g = _c128(gates).copy()
    ps, ph = _c128(psi), _c128(phi)
    fb = np.zeros(L) if record else None
    fa = np.zeros(L) if record else None
    c = load().qd_sweep(d, n, L, _p(pr), _p(kd), ps.shape[0], _p(ps), _p(ph), _p(g), beta, gamma_scale,
                        _p(fb), _p(fa))
    return (g, c, fb, fa) if record else (g, c)


def qd_environment1(d, n, a, b, qa):
    aa, bb = _c128(a), _c128(b)
    G = np.zeros((d, d), dtype=np.complex128)
    load().qd_environment1(d, n, aa.shape[0], _p(aa), _p(bb), qa, _p(G))
    return G


def qd_update_gate1(d, G1, beta=0.0, u=None):
    """v <- polar((1 - beta) G1 + beta v) on the slot u = v (x) I_d (identity slot if None)."""
    uu = np.eye(d * d, dtype=np.complex128) if u is None else _c128(u).copy()
    load().qd_update_gate1(d, _p(_c128(G1)), beta, _p(uu))
    return uu


def qd_haar_gate1(d, seed, start, gate):
    u = np.zeros((d * d, d * d), dtype=np.complex128)
    load().qd_haar_gate1(d, seed, start, gate, _p(u))
    return u


def qd_instantiate(d, n, pairs, psi, phi, n_val=0, params=None, gates_in=None, kinds=None, fixed=None):
    """Qudit instantiation on a fixed sample set (the last n_val rows validate); kinds and
    fixed ([L][d^2][d^2], read for constant gates) as for ``instantiate``."""
    pr = _pairs(pairs)
    L = pr.shape[0]
    kd = _kinds(kinds, L)
    fx = None if fixed is None else _c128(fixed)
    par = Params(**(params or default_params()))
    ps, ph = _c128(psi), _c128(phi)
    gi = None if gates_in is None else _c128(gates_in)
    out = np.zeros((L, d * d, d * d), dtype=np.complex128)
    res = Result()
    rc = load().qd_instantiate(d, n, L, _p(pr), _p(kd), _p(fx), _p(ps), _p(ph), ps.shape[0], n_val,
                               C.byref(par), _p(gi), _p(out), C.byref(res), None)
    if rc != 0:
        raise ValueError(f"qd_instantiate failed: {rc}")
    info = {f: getattr(res, f) for f, _ in Result._fields_}
    info["reason_name"] = REASONS[res.reason]
    return out, info


def qd_draw_states(d, n, M, seed, role, stream):
    """M orthonormal Haar states on d^n amplitudes ([M][d^n], the qubit draw's streams)."""
    out = np.zeros((M, d ** n), dtype=np.complex128)
    rc = load().qd_draw_states(d, n, M, seed, role, stream, _p(out))
    if rc != 0:
        raise ValueError(f"qd_draw_states failed: {rc}")
    return out


def qd_instantiate_target(d, n, pairs, *, U=None, target_pairs=None, target_gates=None,
                          params=None, gates_in=None, trace_capacity=0, doubling_capacity=0,
                          kinds=None, fixed=None):
    """Qudit instantiation against a dense target ``U`` ([d^n][d^n]) or a target circuit
    (``target_pairs`` + ``target_gates`` [Lt][d^2][d^2]), with drawn training and validation
    states. Returns (gates, result dict), with the trace as in ``instantiate``."""
    lib = load()
    pr = _pairs(pairs)
    L, D = pr.shape[0], d * d
    par = Params(**(params or default_params()))
    keep = []
    if U is not None:
        kind = TARGET_DENSE
        Uc = _c128(U)
        keep.append(Uc)
        args = (_p(Uc), 0, None, None)
    else:
        kind = TARGET_CIRCUIT
        tp = _pairs(target_pairs)
        tg = _c128(target_gates)
        keep += [tp, tg]
        args = (None, tp.shape[0], _p(tp), _p(tg))
    gi = None if gates_in is None else _c128(gates_in)
    out = np.zeros((L, D, D), dtype=np.complex128)
    res = Result()
    tr = None
    if trace_capacity or doubling_capacity:
        tr, bufs, dbl = _make_trace(max(trace_capacity, 1), doubling_capacity, par.multistarts
                                    if par.multistarts > 0 else 1, L, D * D, d ** n)
    kd = _kinds(kinds, L)
    fx = None if fixed is None else _c128(fixed)
    rc = lib.qd_instantiate_target(d, n, L, _p(pr), _p(kd), _p(fx), kind, *args, C.byref(par), _p(gi),
                                   _p(out), C.byref(res), C.byref(tr) if tr is not None else None)
    if rc != 0:
        raise ValueError(f"qd_instantiate_target failed: {rc}")
    info = {f: getattr(res, f) for f, _ in Result._fields_}
    info["reason_name"] = REASONS[res.reason]
    if tr is not None:
        info["trace"] = _read_trace(tr, bufs, dbl)
    return out, info


__all__ = [
    "Params", "Result", "ROLE_TRAIN", "ROLE_VAL", "ROLE_INIT", "REASONS", "default_params",
    "philox4x32_10", "cgauss", "ginibre", "orthonormalize", "draw_states", "haar_gate",
    "haar_gate2", "initial_gates", "kron_i2", "GATE_2Q", "GATE_1Q", "GATE_FIXED",
    "apply_gate", "apply_circuit", "dense_apply", "environment", "environment1", "svd4",
    "update_gate", "update_gate1", "qd_apply_gate", "qd_apply_circuit", "qd_environment",
    "qd_svd", "qd_update_gate", "qd_haar_gate", "qd_sweep", "qd_instantiate",
    "qd_draw_states", "qd_instantiate_target", "qd_environment1", "qd_update_gate1", "qd_haar_gate1",
    "state_distance", "sweep", "instantiate", "EV_RUN", "EV_SUCCESS", "EV_OVERTRAINED",
    "EV_NOT_GEN", "EV_PLATEAU", "EV_MAX_ITER",
]
