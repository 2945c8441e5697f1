"""Dense brute-force checker for small n (test infrastructure).

Independent of the oracle: gates act through numpy tensor reshapes (axes = qubits,
qubit 0 first, i.e. most significant), and full-unitary QFactor (Sec. 2.1, Eq. 1 and
Eq. 2) is written on 2^n x 2^n matrices with the environment as a partial trace.
"""
from __future__ import annotations

import numpy as np


def apply_gate_tensor(n, states, a, b, u):
    """Apply 4x4 u on ordered qubits (a, b) to [M][2^n] states via tensor axes."""
    M = states.shape[0]
    t = states.reshape((M,) + (2,) * n)
    t = np.moveaxis(t, (1 + a, 1 + b), (1, 2))
    shp = t.shape
    t = t.reshape(M, 4, -1)
    t = np.einsum("qp,mpr->mqr", u, t)
    t = t.reshape(shp)
    t = np.moveaxis(t, (1, 2), (1 + a, 1 + b))
    return t.reshape(M, -1)


def gate_matrix(n, a, b, u):
    """Full 2^n x 2^n matrix of u on (a, b): its columns are the images of basis states."""
    N = 1 << n
    return apply_gate_tensor(n, np.eye(N, dtype=np.complex128), a, b, u).T


def circuit_matrix(n, pairs, gates):
    N = 1 << n
    C = np.eye(N, dtype=np.complex128)
    for (a, b), u in zip(np.asarray(pairs).reshape(-1, 2), gates):
        C = gate_matrix(n, int(a), int(b), u) @ C
    return C


def full_distance(U, C):
    """Eq. 1 divided by 2^n: ||U - C||_F^2 / 2^n = 2 - 2 Re Tr(U^dag C) / 2^n."""
    N = U.shape[0]
    return float(np.linalg.norm(U - C) ** 2 / N)


def partial_trace_env(n, a, b, X):
    """E[p][q] = sum_r X[(p,r),(q,r)] with the gate's qubits (a, b) as the local index
    (so that Re Tr(X (u (x) I)) = Re Tr(E u))."""
    N = 1 << n
    T = X.reshape((2,) * (2 * n))
    rows = list(range(n))
    cols = list(range(n, 2 * n))
    order = [a, b] + [q for q in rows if q not in (a, b)]
    order += [n + a, n + b] + [n + q for q in rows if q not in (a, b)]
    T = np.transpose(T, order).reshape(4, N // 4, 4, N // 4)
    return np.einsum("prqr->pq", T)


def partial_trace_env1(n, a, X):
    """E[p][q] = sum_r X[(p,r),(q,r)] over the n-1 qubits other than a (2x2)."""
    T = X.reshape((2,) * (2 * n))
    order = [a] + [q for q in range(n) if q != a] + [n + a] + [n + q for q in range(n) if q != a]
    T = np.transpose(T, order).reshape(2, (1 << n) // 2, 2, (1 << n) // 2)
    return np.einsum("prqr->pq", T)


def one_qubit_matrix(n, a, v):
    """Full 2^n x 2^n matrix of the 2x2 v on qubit a: I_{2^a} (x) v (x) I_{2^(n-1-a)}."""
    return np.kron(np.kron(np.eye(1 << a), v), np.eye(1 << (n - 1 - a)))


def polar_unitary(A):
    W, s, Vh = np.linalg.svd(A)
    return W @ Vh


def dense_qfactor_sweep(n, pairs, gates, U, kinds=None):
    """One full-unitary QFactor sweep, right to left (Sec. 2.1): for gate k with
    C = A u_k B, f = Re Tr(U^dag A u_k B) = Re Tr(E u_k), E = Tr_rest(B U^dag A);
    u_k <- Y X^dag for E = X D Y^dag (Eq. 2). A uses already-updated gates.
    kinds (0 two-qubit, 1 one-qubit, 2 fixed): a one-qubit gate's slot is v (x) I_2 and v
    is updated from the 2x2 partial trace over every other qubit; a fixed gate is kept."""
    pairs = np.asarray(pairs).reshape(-1, 2)
    g = [np.array(x, dtype=np.complex128) for x in gates]
    L = len(g)
    N = 1 << n
    for k in range(L - 1, -1, -1):
        A = np.eye(N, dtype=np.complex128)
        for j in range(k + 1, L):
            A = gate_matrix(n, int(pairs[j][0]), int(pairs[j][1]), g[j]) @ A
        B = np.eye(N, dtype=np.complex128)
        for j in range(k):
            B = gate_matrix(n, int(pairs[j][0]), int(pairs[j][1]), g[j]) @ B
        kind = 0 if kinds is None else int(kinds[k])
        if kind == 2:
            continue
        if kind == 1:
            E = partial_trace_env1(n, int(pairs[k][0]), B @ U.conj().T @ A)
            X, d, Yh = np.linalg.svd(E)
            g[k] = np.kron(Yh.conj().T @ X.conj().T, np.eye(2))
            continue
        E = partial_trace_env(n, int(pairs[k][0]), int(pairs[k][1]), B @ U.conj().T @ A)
        X, d, Yh = np.linalg.svd(E)
        g[k] = Yh.conj().T @ X.conj().T
    return np.stack(g)


# ------------------------------------------------------------------------ qudits
def apply_gate_tensor_d(d, n, states, a, b, u):
    """Apply the d^2 x d^2 gate u on ordered qudits (a, b) to [M][d^n] states via tensor
    axes (qudit 0 first)."""
    M = states.shape[0]
    t = states.reshape((M,) + (d,) * n)
    t = np.moveaxis(t, (1 + a, 1 + b), (1, 2))
    shp = t.shape
    t = t.reshape(M, d * d, -1)
    t = np.einsum("qp,mpr->mqr", u, t)
    t = t.reshape(shp)
    t = np.moveaxis(t, (1, 2), (1 + a, 1 + b))
    return t.reshape(M, -1)


def gate_matrix_d(d, n, a, b, u):
    N = d ** n
    return apply_gate_tensor_d(d, n, np.eye(N, dtype=np.complex128), a, b, u).T


def circuit_matrix_d(d, n, pairs, gates):
    C = np.eye(d ** n, dtype=np.complex128)
    for (a, b), u in zip(np.asarray(pairs).reshape(-1, 2), gates):
        C = gate_matrix_d(d, n, int(a), int(b), u) @ C
    return C


def partial_trace_env_d(d, n, a, b, X):
    """E[p][q] = sum_r X[(p,r),(q,r)] with qudits (a, b) as the local index."""
    N = d ** n
    T = X.reshape((d,) * (2 * n))
    rest = [q for q in range(n) if q not in (a, b)]
    order = [a, b] + rest + [n + a, n + b] + [n + q for q in rest]
    T = np.transpose(T, order).reshape(d * d, N // (d * d), d * d, N // (d * d))
    return np.einsum("prqr->pq", T)


def dense_qfactor_sweep_d(d, n, pairs, gates, U):
    """Full-unitary QFactor sweep on qudits (as dense_qfactor_sweep, base-d axes)."""
    pairs = np.asarray(pairs).reshape(-1, 2)
    g = [np.array(x, dtype=np.complex128) for x in gates]
    L = len(g)
    N = d ** n
    for k in range(L - 1, -1, -1):
        A = np.eye(N, dtype=np.complex128)
        for j in range(k + 1, L):
            A = gate_matrix_d(d, n, int(pairs[j][0]), int(pairs[j][1]), g[j]) @ A
        B = np.eye(N, dtype=np.complex128)
        for j in range(k):
            B = gate_matrix_d(d, n, int(pairs[j][0]), int(pairs[j][1]), g[j]) @ B
        E = partial_trace_env_d(d, n, int(pairs[k][0]), int(pairs[k][1]), B @ U.conj().T @ A)
        X, _, Yh = np.linalg.svd(E)
        g[k] = Yh.conj().T @ X.conj().T
    return np.stack(g)
