"""Seeded synthetic problem generators, shared by the tests, the benchmark and the
smoke check.

This module only builds problem *inputs* (circuit templates, target gates, fixed
sample sets for lock-step comparisons). It holds none of the instantiation method's
arithmetic: the states and initial gates that the method itself draws are drawn by
each implementation from its own counter-based generator.

The paper's workloads are partitions of real circuits (U3 + CNOT, 3-12 qubits); they
are not available here, so seeded synthetic circuits of the same sizes stand in:
brickwork and random-pair templates of general two-qubit gates, and U3 + CNOT style
templates of variable one-qubit gates around constant CNOTs, with targets built from
the same template with Haar-random gates, so that an exact solution exists.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014): seed derivation only."""
    x = (x + 0x9E3779B97F4A7C15) & MASK64
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


ROLE_TARGET, ROLE_TRAIN, ROLE_VAL, ROLE_INIT = 0x7A, 0x7B, 0x7C, 0x7D

# Gate kinds of a template: variable two-qubit, variable one-qubit (slot v (x) I_2 on
# (qubit, spectator)), constant.
GATE_2Q, GATE_1Q, GATE_FIXED = 0, 1, 2

# CNOT with the first qubit of the pair as control (local index 2*bit(a) + bit(b)).
CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)


def derive_seed(base: int, problem: int = 0, role: int = ROLE_TARGET, start: int = 0) -> int:
    """seed = SplitMix64(base ^ problem ^ role ^ start), each field in its own bits."""
    return splitmix64((base ^ (problem << 20) ^ (role << 52) ^ (start << 40)) & MASK64)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def linear_template(n: int, repeats: int):
    """Pairs (0,1),(1,2),...,(n-2,n-1) repeated: the 3-qubit workload of 6 gates is
    linear_template(3, 3)."""
    pairs = []
    for _ in range(repeats):
        for q in range(n - 1):
            pairs.append((q, q + 1))
    return np.asarray(pairs, dtype=np.int32)


def brickwork_template(n: int, sublayers: int):
    """Alternating sublayers of nearest-neighbour gates, even pairs (0,1),(2,3),...
    then odd pairs (1,2),(3,4),... . 8 qubits x 6 sublayers = 21 gates; 12 qubits x 8
    sublayers = 44 gates."""
    pairs = []
    for s in range(sublayers):
        first = 0 if s % 2 == 0 else 1
        for q in range(first, n - 1, 2):
            pairs.append((q, q + 1))
    return np.asarray(pairs, dtype=np.int32)


def random_pair_template(n: int, L: int, g: np.random.Generator):
    """L gates on pairs drawn uniformly from the distinct unordered pairs, as (lo, hi)."""
    pairs = []
    for _ in range(L):
        a, b = g.choice(n, size=2, replace=False)
        pairs.append((min(a, b), max(a, b)))
    return np.asarray(pairs, dtype=np.int32).reshape(-1, 2)


def haar_unitary(d: int, g: np.random.Generator):
    """Haar-random d x d unitary for target construction (numpy QR of a complex
    Ginibre matrix with the phases of diag(R) divided out)."""
    z = (g.standard_normal((d, d)) + 1j * g.standard_normal((d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


def haar_gates(L: int, g: np.random.Generator):
    return np.stack([haar_unitary(4, g) for _ in range(L)]) if L else np.zeros((0, 4, 4), complex)


def orthonormal_samples(n: int, M: int, g: np.random.Generator):
    """M orthonormal states of 2^n amplitudes, [M][N], for fixed-sample comparisons."""
    N = 1 << n
    z = (g.standard_normal((N, M)) + 1j * g.standard_normal((N, M))) / np.sqrt(2.0)
    q, _ = np.linalg.qr(z)
    return np.ascontiguousarray(q.T)


def orthonormal_states(N: int, M: int, g: np.random.Generator):
    """M orthonormal states of N amplitudes, [M][N] (numpy QR of a complex Ginibre
    matrix), for qudit sample sets."""
    z = (g.standard_normal((N, M)) + 1j * g.standard_normal((N, M))) / np.sqrt(2.0)
    q, _ = np.linalg.qr(z)
    return np.ascontiguousarray(q.T)


def qudit_brickwork(n: int, sublayers: int):
    """Brickwork pairs of n qudits (as brickwork_template)."""
    return brickwork_template(n, sublayers)


def qudit_circuit_apply(d: int, n: int, states, pairs, gates):
    """Apply d^2 x d^2 gates in order to [M][d^n] states through base-d tensor axes (qudit
    0 first). Input construction only (target sample sets)."""
    out = np.array(states, dtype=np.complex128, copy=True)
    M = out.shape[0]
    for (a, b), u in zip(np.asarray(pairs).reshape(-1, 2), gates):
        t = np.moveaxis(out.reshape((M,) + (d,) * n), (1 + int(a), 1 + int(b)), (1, 2))
        shp = t.shape
        t = np.einsum("qp,mpr->mqr", u, t.reshape(M, d * d, -1)).reshape(shp)
        out = np.moveaxis(t, (1, 2), (1 + int(a), 1 + int(b))).reshape(M, -1)
    return out


def circuit_unitary_columns(n: int, pairs, gates, states):
    """Apply a gate list to [M][N] states by explicit 2^n x 2^n Kronecker embedding.
    Input construction only (used to build fixed target samples); O(4^n) per gate."""
    N = 1 << n
    out = np.array(states, dtype=np.complex128, copy=True)
    for (a, b), u in zip(np.asarray(pairs).reshape(-1, 2), gates):
        full = embed_two_qubit(n, int(a), int(b), u)
        out = out @ full.T
    return out


def embed_two_qubit(n: int, a: int, b: int, u):
    """2^n x 2^n matrix of a 4x4 gate on ordered qubits (a, b), qubit 0 most significant."""
    N = 1 << n
    full = np.zeros((N, N), dtype=np.complex128)
    pa, pb = n - 1 - a, n - 1 - b
    for col in range(N):
        p = 2 * ((col >> pa) & 1) + ((col >> pb) & 1)
        base = col & ~((1 << pa) | (1 << pb))
        for q in range(4):
            row = base | (((q >> 1) & 1) << pa) | ((q & 1) << pb)
            full[row, col] += u[q, p]
    return full


def u3_cnot_template(n: int, sublayers: int):
    """U3 + CNOT style template: a one-qubit gate on every qubit, then brickwork
    sublayers of CNOT blocks, each block a constant CNOT on (q, q+1) followed by one-qubit
    gates on q and q+1 (the shape of synthesised partitions). A one-qubit gate on q names
    spectator (q + 1) mod n. Returns (pairs [L][2], kinds [L], fixed [L][4][4] with the
    CNOTs at the constant gates and the identity elsewhere)."""
    pairs, kinds = [], []
    for q in range(n):
        pairs.append((q, (q + 1) % n))
        kinds.append(GATE_1Q)
    for s in range(sublayers):
        for q in range(s % 2, n - 1, 2):
            pairs += [(q, q + 1), (q, q + 1), (q + 1, q)]
            kinds += [GATE_FIXED, GATE_1Q, GATE_1Q]
    kinds = np.asarray(kinds, dtype=np.int32)
    fixed = np.stack([CNOT if k == GATE_FIXED else np.eye(4, dtype=np.complex128) for k in kinds])
    return np.asarray(pairs, dtype=np.int32), kinds, fixed


def kinds_target_gates(kinds, fixed, g: np.random.Generator):
    """Target gates for a template with gate kinds: Haar 4x4, Haar 2x2 (x) I_2, or the
    constant gate."""
    out = []
    for k, f in zip(kinds, fixed):
        if k == GATE_FIXED:
            out.append(np.array(f, dtype=np.complex128))
        elif k == GATE_1Q:
            out.append(np.kron(haar_unitary(2, g), np.eye(2)))
        else:
            out.append(haar_unitary(4, g))
    return np.stack(out)


# ----------------------------------------------------------------------------------
# Named workloads (sizes of the paper's partitions; synthetic content).
# ----------------------------------------------------------------------------------
def workload_3q(seed_base: int = 0x5A17 + 1):
    """3 qubits, pairs (0,1),(1,2) x 3 (L = 6); target = same template, Haar gates."""
    g = rng(derive_seed(seed_base, 0, ROLE_TARGET))
    pairs = linear_template(3, 3)
    return dict(n=3, pairs=pairs, target_pairs=pairs, target_gates=haar_gates(len(pairs), g))


def workload_brickwork(n: int, sublayers: int, seed_base: int, problem: int = 0):
    g = rng(derive_seed(seed_base, problem, ROLE_TARGET))
    pairs = brickwork_template(n, sublayers)
    return dict(n=n, pairs=pairs, target_pairs=pairs, target_gates=haar_gates(len(pairs), g))


def workload_8q(seed_base: int = 0x5A17 + 2):
    """8-qubit brickwork, 6 sublayers (21 gates)."""
    return workload_brickwork(8, 6, seed_base)


def workload_12q(seed_base: int = 0x5A17 + 3):
    """12-qubit brickwork, 8 sublayers (44 gates)."""
    return workload_brickwork(12, 8, seed_base)


def workload_u3_cnot(n: int, sublayers: int, seed_base: int = 0x5A17 + 6, problem: int = 0):
    """U3 + CNOT style template (u3_cnot_template); target = the same template with Haar
    one-qubit gates and the same CNOTs. 12 qubits x 8 sublayers: 44 CNOTs, 100 one-qubit
    gates."""
    g = rng(derive_seed(seed_base, problem, ROLE_TARGET))
    pairs, kinds, fixed = u3_cnot_template(n, sublayers)
    return dict(n=n, pairs=pairs, kinds=kinds, fixed=fixed, target_pairs=pairs,
                target_gates=kinds_target_gates(kinds, fixed, g))


def batched_u3_cnot_problems(count: int, seed_base: int = 0x5A17 + 10, n_range=(3, 7), sub_range=(1, 4)):
    """Uneven U3 + CNOT problem set: n ~ U{3..7}, brickwork sublayers ~ U{1..4}
    (u3_cnot_template), target = the template with Haar one-qubit gates and the same CNOTs."""
    probs = []
    for pid in range(count):
        g = rng(derive_seed(seed_base, pid, ROLE_TARGET))
        n = int(g.integers(n_range[0], n_range[1] + 1))
        sub = int(g.integers(sub_range[0], sub_range[1] + 1))
        pairs, kinds, fixed = u3_cnot_template(n, sub)
        probs.append(dict(n=n, pairs=pairs, kinds=kinds, fixed=fixed, target_pairs=pairs,
                          target_gates=kinds_target_gates(kinds, fixed, g)))
    return probs


def batched_problems(count: int, seed_base: int = 0x5A17 + 4, n_range=(3, 7), L_range=(2, 20)):
    """Uneven problem set: n ~ U{3..7}, L ~ U{2..20}, random distinct pairs, target =
    the template with Haar gates."""
    probs = []
    for pid in range(count):
        g = rng(derive_seed(seed_base, pid, ROLE_TARGET))
        n = int(g.integers(n_range[0], n_range[1] + 1))
        L = int(g.integers(L_range[0], L_range[1] + 1))
        pairs = random_pair_template(n, L, g)
        probs.append(dict(n=n, pairs=pairs, target_pairs=pairs, target_gates=haar_gates(L, g),
                          seed=derive_seed(seed_base, pid, ROLE_INIT)))
    return probs
