"""GPU tests of the Barrett modular multiplication (tm_mulmod), a consumer
of the high and low products: bit-exact against the oracle's plain
definition on ragged sizes, edge operands, and Fermat's little theorem on
the Mersenne prime 2^521 - 1 through a chain of GPU calls."""
import sys

import numpy as np
import pytest

import oracle
from paper_1703_00640_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _tm():
    import paper_1703_00640_amd as tm
    return tm


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(dev())


def to_host(t):
    return t.cpu().numpy().view(np.uint64)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def modulus(n, seed):
    m = oracle.to_int(inputs.random_limbs(n, seed)) | (1 << (n - 1)) | 1
    return oracle.from_int(m, oracle.nlimbs(n))


def gpu_mulmod(a, b, m, n):
    tm = _tm()
    r = tm.mulmod(to_dev(a), to_dev(b), to_dev(m), to_dev(oracle.barrett_mu(m, n)), n)
    torch.cuda.synchronize()
    return to_host(r)


@pytest.mark.parametrize("n", [2, 3, 63, 64, 65, 127, 521, 1000, 4096, 65537, 1 << 18])
def test_mulmod_random(n):
    say("[mulmod] n=%d" % n)
    m = modulus(n, 11 + n)
    for seed in (1, 2):
        a, b = inputs.operand_pair(n, 600 + seed)
        assert np.array_equal(gpu_mulmod(a, b, m, n), oracle.mulmod(a, b, m, n)), (n, seed)


@pytest.mark.parametrize("n", [2, 64, 129, 3000])
def test_mulmod_edges(n):
    """a = b = m - 1; operands at or above m; zero; m = 2^n - 1 with
    2^(n-1) * 2; the smallest modulus 2^(n-1) + 1."""
    L = oracle.nlimbs(n)
    for m in (modulus(n, n), oracle.from_int((1 << n) - 1, L), oracle.from_int((1 << (n - 1)) + 1, L)):
        M = oracle.to_int(m)
        cases = [(M - 1, M - 1), ((1 << n) - 1, (1 << n) - 1), (M, 5 % (1 << n)), (0, M - 1),
                 (1 << (n - 1), 2)]
        for x, y in cases:
            a, b = oracle.from_int(x, L), oracle.from_int(y, L)
            assert np.array_equal(gpu_mulmod(a, b, m, n), oracle.mulmod(a, b, m, n)), (n, M, x, y)


def test_mulmod_fermat_chain_on_gpu():
    """a^(p-1) = 1 mod p = 2^521 - 1 by square-and-multiply on the GPU, every
    step a tm_mulmod call on device-resident operands."""
    tm = _tm()
    n = 521
    p = (1 << n) - 1
    L = oracle.nlimbs(n)
    m = to_dev(oracle.from_int(p, L))
    mu = to_dev(oracle.barrett_mu(oracle.from_int(p, L), n))
    a = to_dev(oracle.from_int(oracle.to_int(inputs.random_limbs(n, 5)) % p, L))
    r = to_dev(oracle.from_int(1, L))
    ws = torch.empty(tm._load().tm_workspace_bytes_mulmod(n), dtype=torch.uint8, device=dev())
    for bit in bin(p - 1)[2:]:
        r = tm.mulmod(r, r, m, mu, n, workspace=ws)
        if bit == "1":
            r = tm.mulmod(r, a, m, mu, n, workspace=ws)
    torch.cuda.synchronize()
    assert oracle.to_int(to_host(r)) == 1
