"""qfs_environment_noalloc, the entry point for callers that cannot allocate device memory,
against qfs_environment (Sec. 3, Eq. 10) through the C ABI: two calls in a row, the
second on a smaller input, both to FP64 rounding (the two sum in different orders); and its
size limit, checked on the host before any device work."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2405_12866_amd import qfs as Q


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_size_limit_rejected_on_the_host():
    lib = Q.load()
    fake = C.c_void_p(16)  # never dereferenced: the size check comes first
    rc = lib.qfs_environment_noalloc(24, 1 << 8, fake, fake, 0, 1, fake, None)
    assert rc == Q.QFS_EINVAL
    assert "exceeds" in lib.qfs_last_error_detail().decode()
    rc = lib.qfs_environment_noalloc(5, 4, fake, fake, 2, 2, fake, None)
    assert rc == Q.QFS_EINVAL


@pytest.mark.gpu
def test_noalloc_environment_matches_qfs_environment_twice():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = "cuda:0"
    g = np.random.default_rng(2024)
    out = torch.zeros((4, 4), dtype=torch.complex128, device=dev)
    for n, M, qa, qb in ((10, 64, 3, 7), (6, 5, 5, 0)):
        say(f"noalloc environment n={n} M={M} qubits=({qa},{qb})")
        N = 1 << n
        a = torch.as_tensor((g.standard_normal((M, N)) + 1j * g.standard_normal((M, N))) / np.sqrt(N)).to(dev)
        b = torch.as_tensor((g.standard_normal((M, N)) + 1j * g.standard_normal((M, N))) / np.sqrt(N)).to(dev)
        ref = Q.qfs_environment(n, a, b, qa, qb)
        Q.qfs_environment_noalloc(n, a, b, qa, qb, out)
        torch.cuda.synchronize()
        got, want = out.cpu().numpy(), ref.cpu().numpy()
        assert np.max(np.abs(got - want)) <= 1e-12 * max(np.max(np.abs(want)), 1e-300), (n, M, got, want)
