"""Python binding of libqfs_hip.so (the C ABI in include/qfs.h).

Argument marshalling only: every step runs in the HIP library. Device buffers are
torch complex128 tensors on a ROCm device (interleaved re/im doubles, the layout of
qfs_c128); work is issued on torch's current stream. The functions keep the C names.
There is no CPU fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqfs_hip.so")
_lib = None
_lock = threading.Lock()

QFS_OK, QFS_EINVAL, QFS_ENOMEM, QFS_EDEVICE, QFS_EUNSUPPORTED, QFS_ENUMERIC = range(6)
QFS_TARGET_DENSE, QFS_TARGET_CIRCUIT, QFS_TARGET_SAMPLES = 0, 1, 2
QFS_PREC_FP64, QFS_PREC_MIXED = 0, 1
QFS_GATE_2Q, QFS_GATE_1Q, QFS_GATE_FIXED = 0, 1, 2
QFS_BWD_GROUPED, QFS_BWD_PER_GATE = 0, 1
REASONS = {0: "SUCCESS", 1: "PLATEAU", 2: "MAX_ITER", 3: "NOT_GENERALIZED", 4: "TIMEOUT"}


class QfsError(RuntimeError):
    def __init__(self, code, where):
        lib = load()
        super().__init__(f"{where}: {lib.qfs_strerror(code).decode()} ({code}): "
                         f"{lib.qfs_last_error_detail().decode()}")
        self.code = code


class Template(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_gates", C.c_int32), ("pairs", C.POINTER(C.c_int32)),
                ("kinds", C.POINTER(C.c_int32)), ("fixed_gates", C.c_void_p)]


class Target(C.Structure):
    _fields_ = [("kind", C.c_int32), ("U", C.c_void_p), ("circuit", C.POINTER(Template)),
                ("circuit_gates", C.c_void_p), ("psi", C.c_void_p), ("phi", C.c_void_p),
                ("n_samples", C.c_int32), ("n_val", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("dist_tol", C.c_double), ("diff_tol_r", C.c_double),
                ("plateau_window", C.c_int32), ("min_iter", C.c_int32), ("max_iter", C.c_int64),
                ("m_init", C.c_int32), ("m_max", C.c_int32), ("overtrain_ratio", C.c_double),
                ("multistarts", C.c_int32), ("beta", C.c_double), ("seed", C.c_uint64),
                ("fixed_m", C.c_int32), ("m_val", C.c_int32), ("precision", C.c_int32),
                ("refine_below", C.c_double), ("device_mem_budget", C.c_uint64),
                ("time_budget_s", C.c_double), ("hip_stream", C.c_void_p),
                ("timing", C.c_int32), ("batch_sweeps", C.c_int32), ("batch_threads", C.c_int32),
                ("graphs", C.c_int32), ("full_unitary", C.c_int32),
                ("beta_normalized", C.c_int32), ("backward_mode", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("reason", C.c_int32), ("m_final", C.c_int32), ("sweeps", C.c_int32),
                ("restarts", C.c_int32), ("best_start", C.c_int32), ("m_total", C.c_int32),
                ("start_groups", C.c_int32), ("refined", C.c_int32), ("c_train", C.c_double),
                ("c_val", C.c_double), ("seconds", C.c_double), ("start_sweeps", C.c_int64),
                ("sweep_seconds", C.c_double), ("kernel_launches", C.c_int64 * 4),
                ("kernel_seconds", C.c_double * 4), ("kernel_bytes", C.c_double * 4),
                ("m_predicted", C.c_int32), ("starts_run", C.c_int32), ("fallback", C.c_int32),
                ("amp_updates", C.c_double)]


EXPORTS = ["qfs_strerror", "qfs_last_error_detail", "qfs_version", "qfs_release_device_cache",
           "qfs_default_params",
           "qfs_instantiate", "qfs_instantiate_batch", "qfs_instantiate_samples", "qfs_draw_states", "qfs_haar_gates",
           "qfs_apply_gates", "qfs_dense_apply", "qfs_environment", "qfs_environment_noalloc",
           "qfs_polar_update",
           "qfs_sweep", "qfs_state_distance", "qfs_label_batch", "qfs_features",
           "qfs_mlp_num_params", "qfs_mlp_init", "qfs_mlp_get", "qfs_mlp_set", "qfs_mlp_save",
           "qfs_mlp_load", "qfs_mlp_forward", "qfs_mlp_grad", "qfs_mlp_train", "qfs_predict_m",
           "qfs_predict_batch", "qfs_instantiate_learned", "qfs_instantiate_batch_learned",
           "qfs_instantiate_batch_ex", "qfs_qudit_instantiate", "qfs_qudit_instantiate_target",
           "qfs_qudit_instantiate_batch", "qfs_qudit_sweep"]


def load():
    """Load libqfs_hip.so (built by paper_2405_12866_amd.build); raises if absent."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                              "(hipcc --offload-arch=gfx950) first")
        # The library and PyTorch must share one HIP runtime (the library's arguments are
        # torch's device pointers): load torch's first, so that the library's dependency on
        # libamdhip64 resolves to it. Loaded the other way round, the second runtime finds
        # no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = C.CDLL(LIB_PATH)
        P, I32, U32, U64, D = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64, C.c_double
        lib.qfs_strerror.restype = C.c_char_p
        lib.qfs_strerror.argtypes = [C.c_int]
        lib.qfs_last_error_detail.restype = C.c_char_p
        lib.qfs_version.restype = C.c_char_p
        lib.qfs_release_device_cache.argtypes = [C.POINTER(C.c_size_t)]
        lib.qfs_default_params.argtypes = [C.POINTER(Params)]
        lib.qfs_instantiate.argtypes = [C.POINTER(Template), C.POINTER(Target), C.POINTER(Params),
                                        P, P, C.POINTER(Result)]
        lib.qfs_instantiate_batch.argtypes = [I32, C.POINTER(Template), C.POINTER(Target),
                                              C.POINTER(Params), C.POINTER(C.c_void_p),
                                              C.POINTER(Result)]
        lib.qfs_instantiate_samples.argtypes = [C.POINTER(Template), P, P, I32, D, P,
                                                C.POINTER(C.c_double)]
        lib.qfs_draw_states.argtypes = [I32, I32, U64, U32, U32, P, P]
        lib.qfs_haar_gates.argtypes = [U64, I32, I32, P, P]
        lib.qfs_apply_gates.argtypes = [I32, I32, P, I32, P, P, I32, P]
        lib.qfs_dense_apply.argtypes = [I32, I32, P, P, P, P]
        lib.qfs_environment.argtypes = [I32, I32, P, P, I32, I32, P, P]
        lib.qfs_environment_noalloc.argtypes = [I32, I32, P, P, I32, I32, P, P]
        lib.qfs_polar_update.argtypes = [I32, P, D, P, P]
        lib.qfs_sweep.argtypes = [I32, I32, P, P, I32, P, P, I32, P, I32, D, I32, P, P]
        lib.qfs_state_distance.argtypes = [I32, I32, P, P, C.POINTER(C.c_double), P]
        batch_args = [I32, C.POINTER(Template), C.POINTER(Target), C.POINTER(Params)]
        lib.qfs_label_batch.argtypes = batch_args + [P, C.POINTER(Result)]
        lib.qfs_instantiate_batch_ex.argtypes = batch_args + [P, P, C.POINTER(C.c_void_p),
                                                              C.POINTER(Result)]
        lib.qfs_instantiate_batch_learned.argtypes = batch_args + [C.POINTER(C.c_void_p),
                                                                   C.POINTER(Result)]
        lib.qfs_instantiate_learned.argtypes = [C.POINTER(Template), C.POINTER(Target),
                                                C.POINTER(Params), P, C.POINTER(Result)]
        lib.qfs_features.argtypes = [C.POINTER(Template), P]
        lib.qfs_mlp_init.argtypes = [U64]
        lib.qfs_mlp_get.argtypes = [P]
        lib.qfs_mlp_set.argtypes = [P]
        lib.qfs_mlp_save.argtypes = [C.c_char_p]
        lib.qfs_mlp_load.argtypes = [C.c_char_p]
        lib.qfs_mlp_forward.argtypes = [I32, P, P, P]
        lib.qfs_mlp_grad.argtypes = [I32, P, P, P, P, P]
        lib.qfs_mlp_train.argtypes = [I32, P, P, I32, I32, C.c_float, U64, P, P]
        lib.qfs_predict_m.argtypes = [C.POINTER(Template), C.POINTER(Params), P, P]
        lib.qfs_predict_batch.argtypes = [I32, C.POINTER(Template), C.POINTER(Params), P, P]
        lib.qfs_qudit_instantiate.argtypes = [I32, C.POINTER(Template), P, P, I32, I32,
                                              C.POINTER(Params), P, P, C.POINTER(Result)]
        lib.qfs_qudit_instantiate_target.argtypes = [I32, C.POINTER(Template), C.POINTER(Target),
                                                     C.POINTER(Params), P, P, C.POINTER(Result)]
        lib.qfs_qudit_sweep.argtypes = [I32, I32, I32, P, P, I32, P, P, I32, P, I32, D, P, P]
        lib.qfs_qudit_instantiate_batch.argtypes = [I32, I32, C.POINTER(Template), C.POINTER(Target),
                                                    C.POINTER(Params), C.POINTER(C.c_void_p),
                                                    C.POINTER(Result)]
        for name in EXPORTS:
            if name not in ("qfs_strerror", "qfs_last_error_detail", "qfs_version",
                            "qfs_default_params"):
                getattr(lib, name).restype = C.c_int
        _lib = lib
        return lib


def _check(code, where):
    if code != QFS_OK:
        raise QfsError(code, where)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_c128(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128):
        raise TypeError(f"{name} must be a complex128 tensor on a HIP device")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _pairs(pairs):
    import numpy as np
    arr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    return arr, arr.ctypes.data_as(C.POINTER(C.c_int32))


def _template(n, pairs, keep, kinds=None, fixed_gates=None):
    """A Template for ``pairs``; ``kinds`` (per gate QFS_GATE_*) and ``fixed_gates``
    (device [L, 4, 4], read at the constant gates) are optional."""
    import numpy as np
    arr, pp = _pairs(pairs)
    keep.append(arr)
    t = Template(n, arr.shape[0], pp)
    if kinds is not None:
        k = np.ascontiguousarray(np.asarray(kinds, dtype=np.int32).reshape(-1))
        if k.shape[0] != arr.shape[0]:
            raise ValueError("kinds needs one entry per gate")
        keep.append(k)
        t.kinds = k.ctypes.data_as(C.POINTER(C.c_int32))
    if fixed_gates is not None:
        t.fixed_gates = _dev_c128(fixed_gates, "fixed_gates")
    return t


def qfs_default_params(**overrides) -> dict:
    p = Params()
    load().qfs_default_params(C.byref(p))
    d = {f: getattr(p, f) for f, _ in Params._fields_ if f != "hip_stream"}
    for k, v in overrides.items():
        if k not in d:
            raise KeyError(k)
        d[k] = v
    return d


def _params(d):
    p = Params()
    load().qfs_default_params(C.byref(p))
    for k, v in (d or {}).items():
        setattr(p, k, v)
    p.hip_stream = _stream()
    return p


def _fill_target(tgt, n, keep, U=None, target_pairs=None, target_gates=None, psi=None,
                 phi=None, n_val=0):
    """Fill a Target from one target form; returns the device of its tensors."""
    if U is not None:
        tgt.kind = QFS_TARGET_DENSE
        tgt.U = _dev_c128(U, "U")
        return U.device
    if target_pairs is not None:
        tarr, tp = _pairs(target_pairs)
        ct = Template(n, tarr.shape[0], tp)
        keep += [tarr, ct]
        tgt.kind = QFS_TARGET_CIRCUIT
        tgt.circuit = C.pointer(ct)
        tgt.circuit_gates = _dev_c128(target_gates, "target_gates")
        return target_gates.device
    tgt.kind = QFS_TARGET_SAMPLES
    tgt.psi = _dev_c128(psi, "psi")
    tgt.phi = _dev_c128(phi, "phi")
    tgt.n_samples = psi.shape[0]
    tgt.n_val = n_val
    return psi.device


def _info(res):
    info = {f: getattr(res, f) for f, _ in Result._fields_}
    for f in ("kernel_launches", "kernel_seconds", "kernel_bytes"):
        info[f] = list(info[f])
    info["reason_name"] = REASONS.get(res.reason, "?")
    return info


def _single(fn_name, n, pairs, params, gates_in, target, kinds=None, fixed_gates=None):
    import torch
    lib = load()
    keep = []
    tmpl = _template(n, pairs, keep, kinds, fixed_gates)
    L = tmpl.n_gates
    tgt = Target()
    dev = _fill_target(tgt, n, keep, **target)
    par = _params(params)
    out = torch.empty((L, 4, 4), dtype=torch.complex128, device=dev)
    res = Result()
    if fn_name == "qfs_instantiate":
        gi = _dev_c128(gates_in, "gates_in") if gates_in is not None else None
        rc = lib.qfs_instantiate(C.byref(tmpl), C.byref(tgt), C.byref(par), gi,
                                 C.c_void_p(out.data_ptr()), C.byref(res))
    else:
        rc = lib.qfs_instantiate_learned(C.byref(tmpl), C.byref(tgt), C.byref(par),
                                         C.c_void_p(out.data_ptr()), C.byref(res))
    _check(rc, fn_name)
    return out, _info(res)


def qfs_instantiate(n, pairs, *, U=None, target_pairs=None, target_gates=None, psi=None,
                    phi=None, n_val=0, params=None, gates_in=None, kinds=None, fixed_gates=None):
    """QFactor-Sample instantiation on the device. Exactly one target form: dense ``U``
    [N, N]; a circuit (``target_pairs``, ``target_gates`` [Lt, 4, 4]); or samples
    ``psi``/``phi`` [n_samples, N] whose last ``n_val`` rows validate. ``kinds`` (per gate
    QFS_GATE_2Q / QFS_GATE_1Q / QFS_GATE_FIXED) and ``fixed_gates`` (device [L, 4, 4])
    describe templates with one-qubit and constant gates. Returns (gates [L, 4, 4]
    complex128 device tensor, result dict)."""
    return _single("qfs_instantiate", n, pairs, params, gates_in,
                   dict(U=U, target_pairs=target_pairs, target_gates=target_gates, psi=psi,
                        phi=phi, n_val=n_val), kinds, fixed_gates)


def qfs_instantiate_learned(n, pairs, *, U=None, target_pairs=None, target_gates=None,
                            psi=None, phi=None, n_val=0, params=None):
    """qfs_instantiate from the predicted initial M and start count, with the plain
    method as fallback. Needs loaded network weights (qfs_mlp_load / qfs_mlp_set)."""
    return _single("qfs_instantiate_learned", n, pairs, params, None,
                   dict(U=U, target_pairs=target_pairs, target_gates=target_gates, psi=psi,
                        phi=phi, n_val=n_val))


_TARGET_KEYS = ("U", "target_pairs", "target_gates", "psi", "phi", "n_val")


def _batch(fn_name, problems, params, with_gates=True, per_problem=None):
    import numpy as np
    import torch
    lib = load()
    P = len(problems)
    tmpls = (Template * P)()
    tgts = (Target * P)()
    keep, outs = [], []
    for i, pr in enumerate(problems):
        tmpls[i] = _template(pr["n"], pr["pairs"], keep, pr.get("kinds"), pr.get("fixed_gates"))
        dev = _fill_target(tgts[i], pr["n"], keep, **{k: pr[k] for k in _TARGET_KEYS if k in pr})
        if with_gates:
            outs.append(torch.empty((tmpls[i].n_gates, 4, 4), dtype=torch.complex128, device=dev))
    res = (Result * P)()
    par = _params(params)
    if with_gates:
        ptrs = (C.c_void_p * P)(*[o.data_ptr() for o in outs])
        extra = []
        if per_problem is not None:
            arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.int32) for a in per_problem]
            keep += arrs
            extra = [None if a is None else a.ctypes.data_as(C.c_void_p) for a in arrs]
        _check(getattr(lib, fn_name)(P, tmpls, tgts, C.byref(par), *extra, ptrs, res), fn_name)
        return outs, [_info(r) for r in res]
    succ = np.zeros(P, dtype=np.int32)
    _check(getattr(lib, fn_name)(P, tmpls, tgts, C.byref(par), succ.ctypes.data_as(C.c_void_p),
                                 res), fn_name)
    return succ, [_info(r) for r in res]


def qfs_instantiate_batch(problems, params=None):
    """Batched instantiation. ``problems``: list of dicts with ``n``, ``pairs`` and one
    target form (``U``; ``target_pairs`` + ``target_gates``; or ``psi``/``phi`` with
    ``n_val``), device tensors as in qfs_instantiate. Problem p uses seed
    params["seed"] + p. Returns (list of gate tensors [L, 4, 4], list of result dicts)."""
    return _batch("qfs_instantiate_batch", problems, params)


def qfs_instantiate_batch_ex(problems, params=None, m_init=None, starts=None):
    """qfs_instantiate_batch with optional per-problem initial M and start counts."""
    return _batch("qfs_instantiate_batch_ex", problems, params, per_problem=(m_init, starts))


def qfs_instantiate_batch_learned(problems, params=None):
    """qfs_instantiate_batch with predicted initial M and start counts per problem and a
    batched plain rerun of the problems that did not succeed."""
    return _batch("qfs_instantiate_batch_learned", problems, params)


def qfs_label_batch(problems, params=None):
    """Every start of every problem run to its own stop at fixed M = params["m_init"].
    Returns (successful starts per problem as an int32 array, result dicts)."""
    return _batch("qfs_label_batch", problems, params, with_gates=False)


def qfs_features(n, pairs):
    """The 64 structural features of a template (host computation in the library)."""
    import numpy as np
    arr, pp = _pairs(pairs)
    out = np.zeros(64, dtype=np.float32)
    tmpl = Template(n, arr.shape[0], pp)
    _check(load().qfs_features(C.byref(tmpl), out.ctypes.data_as(C.c_void_p)), "qfs_features")
    return out


def qfs_release_device_cache():
    """Free the device buffers the library keeps between calls; returns the bytes freed."""
    freed = C.c_size_t(0)
    _check(load().qfs_release_device_cache(C.byref(freed)), "qfs_release_device_cache")
    return freed.value


def qfs_mlp_num_params():
    return load().qfs_mlp_num_params()


def qfs_mlp_init(seed):
    _check(load().qfs_mlp_init(seed), "qfs_mlp_init")


def qfs_mlp_get():
    import numpy as np
    out = np.zeros(qfs_mlp_num_params(), dtype=np.float32)
    _check(load().qfs_mlp_get(out.ctypes.data_as(C.c_void_p)), "qfs_mlp_get")
    return out


def qfs_mlp_set(params):
    import numpy as np
    arr = np.ascontiguousarray(params, dtype=np.float32)
    if arr.size != qfs_mlp_num_params():
        raise ValueError("wrong parameter count")
    _check(load().qfs_mlp_set(arr.ctypes.data_as(C.c_void_p)), "qfs_mlp_set")


def qfs_mlp_save(path):
    _check(load().qfs_mlp_save(os.fsencode(path)), "qfs_mlp_save")


def qfs_mlp_load(path):
    _check(load().qfs_mlp_load(os.fsencode(path)), "qfs_mlp_load")


def _dev_f32(t, name, cols):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous() and t.dim() == 2 and t.shape[1] == cols):
        raise TypeError(f"{name} must be a contiguous float32 [count, {cols}] tensor on a HIP device")
    return C.c_void_p(t.data_ptr())


def qfs_mlp_forward(features):
    import torch
    out = torch.empty((features.shape[0], 2), dtype=torch.float32, device=features.device)
    _check(load().qfs_mlp_forward(features.shape[0], _dev_f32(features, "features", 64),
                                  C.c_void_p(out.data_ptr()), _stream()), "qfs_mlp_forward")
    return out


def qfs_mlp_grad(features, targets):
    """Returns (gradient as a float32 numpy array, mean loss)."""
    import numpy as np
    g = np.zeros(qfs_mlp_num_params(), dtype=np.float32)
    loss = C.c_float()
    _check(load().qfs_mlp_grad(features.shape[0], _dev_f32(features, "features", 64),
                               _dev_f32(targets, "targets", 2), g.ctypes.data_as(C.c_void_p),
                               C.byref(loss), _stream()), "qfs_mlp_grad")
    return g, loss.value


def qfs_mlp_train(features, targets, epochs, batch, lr, seed=0):
    """Returns the per-epoch mean mini-batch loss (numpy)."""
    import numpy as np
    out = np.zeros(epochs, dtype=np.float32)
    _check(load().qfs_mlp_train(features.shape[0], _dev_f32(features, "features", 64),
                                _dev_f32(targets, "targets", 2), epochs, batch, lr, seed,
                                out.ctypes.data_as(C.c_void_p), _stream()), "qfs_mlp_train")
    return out


def qfs_predict_m(n, pairs, params=None):
    """Returns (predicted initial M, keep mask over starts)."""
    arr, pp = _pairs(pairs)
    tmpl = Template(n, arr.shape[0], pp)
    m0 = C.c_int32()
    mask = C.c_uint32()
    _check(load().qfs_predict_m(C.byref(tmpl), C.byref(_params(params)), C.byref(m0),
                                C.byref(mask)), "qfs_predict_m")
    return m0.value, mask.value


def qfs_predict_batch(templates, params=None):
    """templates: list of (n, pairs). Returns (M0 array, start-count array)."""
    import numpy as np
    P = len(templates)
    tmpls = (Template * P)()
    keep = []
    for i, (n, pairs) in enumerate(templates):
        arr, pp = _pairs(pairs)
        keep.append(arr)
        tmpls[i] = Template(n, arr.shape[0], pp)
    m0 = np.zeros(P, dtype=np.int32)
    k = np.zeros(P, dtype=np.int32)
    _check(load().qfs_predict_batch(P, tmpls, C.byref(_params(params)),
                                    m0.ctypes.data_as(C.c_void_p), k.ctypes.data_as(C.c_void_p)),
           "qfs_predict_batch")
    return m0, k


def qfs_instantiate_samples(n, pairs, psi, phi, M, tol):
    import torch
    arr, pp = _pairs(pairs)
    tmpl = Template(n, arr.shape[0], pp)
    out = torch.empty((arr.shape[0], 4, 4), dtype=torch.complex128, device=psi.device)
    cost = C.c_double()
    _check(load().qfs_instantiate_samples(C.byref(tmpl), _dev_c128(psi, "psi"),
                                          _dev_c128(phi, "phi"), M, tol,
                                          C.c_void_p(out.data_ptr()), C.byref(cost)),
           "qfs_instantiate_samples")
    return out, cost.value


def qfs_draw_states(n, M, seed, role=1, stream=0, device="cuda"):
    import torch
    out = torch.empty((M, 1 << n), dtype=torch.complex128, device=device)
    _check(load().qfs_draw_states(n, M, seed, role, stream, C.c_void_p(out.data_ptr()), _stream()),
           "qfs_draw_states")
    return out


def qfs_haar_gates(seed, starts, L, device="cuda"):
    import torch
    out = torch.empty((starts, L, 4, 4), dtype=torch.complex128, device=device)
    _check(load().qfs_haar_gates(seed, starts, L, C.c_void_p(out.data_ptr()), _stream()),
           "qfs_haar_gates")
    return out


def qfs_apply_gates(n, states, pairs, gates, dagger=False):
    """In place on ``states`` [M, N]; returns it."""
    arr, pp = _pairs(pairs)
    _check(load().qfs_apply_gates(n, states.shape[0], _dev_c128(states, "states"), arr.shape[0],
                                  pp, _dev_c128(gates, "gates"), 1 if dagger else 0, _stream()),
           "qfs_apply_gates")
    return states


def qfs_dense_apply(n, U, psi):
    import torch
    out = torch.empty_like(psi)
    _check(load().qfs_dense_apply(n, psi.shape[0], _dev_c128(U, "U"), _dev_c128(psi, "psi"),
                                  C.c_void_p(out.data_ptr()), _stream()), "qfs_dense_apply")
    return out


def qfs_environment(n, a, b, qa, qb):
    import torch
    g = torch.empty((4, 4), dtype=torch.complex128, device=a.device)
    _check(load().qfs_environment(n, a.shape[0], _dev_c128(a, "a"), _dev_c128(b, "b"), qa, qb,
                                  C.c_void_p(g.data_ptr()), _stream()), "qfs_environment")
    return g


def qfs_environment_noalloc(n, a, b, qa, qb, gamma):
    """Into the caller's device tensor ``gamma`` [4, 4] complex128 (the library allocates
    nothing); stream-ordered on the current stream."""
    _check(load().qfs_environment_noalloc(n, a.shape[0], _dev_c128(a, "a"), _dev_c128(b, "b"), qa, qb,
                                          _dev_c128(gamma, "gamma"), _stream()), "qfs_environment_noalloc")
    return gamma


def qfs_polar_update(gamma, beta=0.0, u=None):
    """gamma [count, 4, 4]; returns the updated gates (a new tensor unless ``u`` given)."""
    import torch
    count = gamma.shape[0]
    if u is None:
        u = torch.zeros_like(gamma)
    _check(load().qfs_polar_update(count, _dev_c128(gamma, "gamma"), beta, _dev_c128(u, "u"),
                                   _stream()), "qfs_polar_update")
    return u


def qfs_sweep(n, pairs, psi, phi, gates, precision=QFS_PREC_FP64, beta=0.0, kinds=None,
              backward=None):
    """One sweep of ``gates`` [starts, L, 4, 4] (updated in place); returns c_train list.
    ``kinds``: per-gate QFS_GATE_* (constant gates are their own entries). ``backward``:
    QFS_BWD_GROUPED (default) or QFS_BWD_PER_GATE."""
    import numpy as np
    arr, pp = _pairs(pairs)
    starts = gates.shape[0]
    c = np.zeros(starts)
    kd = None
    if kinds is not None:
        kd = np.ascontiguousarray(np.asarray(kinds, dtype=np.int32).reshape(-1))
        if kd.shape[0] != arr.shape[0]:
            raise ValueError("kinds needs one entry per gate")
    _check(load().qfs_sweep(n, arr.shape[0], pp, None if kd is None else kd.ctypes.data_as(C.c_void_p),
                            psi.shape[0], _dev_c128(psi, "psi"),
                            _dev_c128(phi, "phi"), starts, _dev_c128(gates, "gates"), precision,
                            beta, QFS_BWD_GROUPED if backward is None else backward,
                            c.ctypes.data_as(C.c_void_p), _stream()), "qfs_sweep")
    return c


def qfs_qudit_sweep(d, n, pairs, psi, phi, gates, precision=QFS_PREC_FP64, beta=0.0, kinds=None):
    """One qudit sweep of ``gates`` [starts, L, d^2, d^2] (in place); returns c_train.
    ``kinds``: per-gate QFS_GATE_* (constant gates are their own entries)."""
    import numpy as np
    arr, pp = _pairs(pairs)
    starts = gates.shape[0]
    c = np.zeros(starts)
    kd = None
    if kinds is not None:
        kd = np.ascontiguousarray(np.asarray(kinds, dtype=np.int32).reshape(-1))
        if kd.shape[0] != arr.shape[0]:
            raise ValueError("kinds needs one entry per gate")
    _check(load().qfs_qudit_sweep(d, n, arr.shape[0], pp, None if kd is None else kd.ctypes.data_as(C.c_void_p),
                                  psi.shape[0], _dev_c128(psi, "psi"),
                                  _dev_c128(phi, "phi"), starts, _dev_c128(gates, "gates"), precision,
                                  beta, c.ctypes.data_as(C.c_void_p), _stream()), "qfs_qudit_sweep")
    return c


def qfs_qudit_instantiate(d, n, pairs, psi, phi, n_val=0, params=None, gates_in=None, kinds=None,
                          fixed_gates=None):
    """Qudit instantiation on a fixed sample set ``psi``/``phi`` [n_samples, d^n] whose last
    ``n_val`` rows validate; ``kinds`` and ``fixed_gates`` (device [L, d^2, d^2]) as for
    qubits. Returns (gates [L, d^2, d^2] device tensor, result dict)."""
    import torch
    keep = []
    tmpl = _template(n, pairs, keep, kinds, fixed_gates)
    out = torch.empty((tmpl.n_gates, d * d, d * d), dtype=torch.complex128, device=psi.device)
    par = _params(params)
    res = Result()
    gi = _dev_c128(gates_in, "gates_in") if gates_in is not None else None
    _check(load().qfs_qudit_instantiate(d, C.byref(tmpl), _dev_c128(psi, "psi"), _dev_c128(phi, "phi"),
                                        psi.shape[0], n_val, C.byref(par), gi,
                                        C.c_void_p(out.data_ptr()), C.byref(res)), "qfs_qudit_instantiate")
    return out, _info(res)


def qfs_qudit_instantiate_target(d, n, pairs, *, U=None, target_pairs=None, target_gates=None,
                                 psi=None, phi=None, n_val=0, params=None, gates_in=None, kinds=None,
                                 fixed_gates=None):
    """Qudit instantiation with one target form: dense ``U`` [d^n, d^n] or a circuit
    (``target_pairs``, ``target_gates`` [Lt, d^2, d^2]) with states drawn on the device, or
    samples ``psi``/``phi``; ``kinds`` and ``fixed_gates`` as for qubits. Returns (gates
    [L, d^2, d^2] device tensor, result dict)."""
    import torch
    keep = []
    tmpl = _template(n, pairs, keep, kinds, fixed_gates)
    tgt = Target()
    dev = _fill_target(tgt, n, keep, U=U, target_pairs=target_pairs, target_gates=target_gates,
                       psi=psi, phi=phi, n_val=n_val)
    out = torch.empty((tmpl.n_gates, d * d, d * d), dtype=torch.complex128, device=dev)
    par = _params(params)
    res = Result()
    gi = _dev_c128(gates_in, "gates_in") if gates_in is not None else None
    _check(load().qfs_qudit_instantiate_target(d, C.byref(tmpl), C.byref(tgt), C.byref(par), gi,
                                               C.c_void_p(out.data_ptr()), C.byref(res)),
           "qfs_qudit_instantiate_target")
    return out, _info(res)


def qfs_qudit_instantiate_batch(d, problems, params=None):
    """Qudit problems side by side: ``problems`` is a list of dicts with n, pairs, optional
    kinds / fixed_gates, and one target form (U; target_pairs + target_gates; psi + phi +
    n_val). Returns (list of gates [L, d^2, d^2] device tensors, list of result dicts)."""
    import torch
    P = len(problems)
    keep = []
    tmpls = (Template * P)()
    tgts = (Target * P)()
    outs = []
    dev = None
    for i, pr in enumerate(problems):
        tmpls[i] = _template(pr["n"], pr["pairs"], keep, pr.get("kinds"), pr.get("fixed_gates"))
        dev = _fill_target(tgts[i], pr["n"], keep, **{k: pr[k] for k in _TARGET_KEYS if k in pr})
        outs.append(torch.empty((tmpls[i].n_gates, d * d, d * d), dtype=torch.complex128, device=dev))
    ptrs = (C.c_void_p * P)(*[o.data_ptr() for o in outs])
    res = (Result * P)()
    par = _params(params)
    _check(load().qfs_qudit_instantiate_batch(d, P, tmpls, tgts, C.byref(par), ptrs, res),
           "qfs_qudit_instantiate_batch")
    return outs, [_info(r) for r in res]


def qfs_state_distance(n, x, y):
    out = C.c_double()
    _check(load().qfs_state_distance(n, x.shape[0], _dev_c128(x, "x"), _dev_c128(y, "y"),
                                     C.byref(out), _stream()), "qfs_state_distance")
    return out.value
