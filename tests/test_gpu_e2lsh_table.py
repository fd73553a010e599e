"""GPU parity of the E2LSH table's near-neighbour lists (the E2LSH class's
get_near_neighbours; Sec. "Random Projection", "Boosting the Probability")
against the oracle: offsets and lists bit-exact, including their order."""
import numpy as np
import pytest

import synth
from tests.gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stag():
    import torch
    assert torch.cuda.is_available()
    import paper_2407_07096_amd as s
    s.load()
    return s


def _compare(stag, orc, X, Q, K, L, seed):
    import torch
    d = X.shape[1]
    G, b = synth.e2lsh_randomness(K * L, d, seed)
    t = stag.E2LSHTable(to_dev(X), to_dev(G), to_dev(b), K, L)
    off, idx = t.near_neighbours(to_dev(Q))
    off2, idx2 = t.near_neighbours(to_dev(Q))
    torch.cuda.synchronize()
    t.close()
    off_ref, idx_ref = orc.e2lsh_near_neighbours(X, Q, G, b, K, L)
    assert np.array_equal(off.cpu().numpy(), off_ref)
    assert np.array_equal(idx.cpu().numpy(), idx_ref)
    assert torch.equal(off, off2) and torch.equal(idx, idx2)
    return off_ref, idx_ref


def test_config1_lists(stag, orc):
    X, Q, _ = synth.config_points(1)
    announce("e2lsh table config1 n=m=1000 d=10 K=8 L=16")
    off, _ = _compare(stag, orc, X, Q, 8, 16, 3001)
    assert off[-1] > 0


def test_self_queries_list_themselves(stag, orc):
    X, _, _ = synth.config_points(1)
    announce("e2lsh table Q = X")
    off, idx = _compare(stag, orc, X, X, 8, 16, 3001)
    assert all(i in idx[off[i]:off[i + 1]] for i in range(X.shape[0]))


@pytest.mark.parametrize("n,m,d,K,L", [(1, 1, 1, 1, 1), (37, 5, 3, 2, 3), (3000, 129, 64, 6, 20),
                                       (5000, 64, 100, 4, 64), (2000, 50, 784, 3, 8), (4099, 65, 17, 1, 33)])
def test_ragged_shapes(stag, orc, n, m, d, K, L):
    rng = np.random.default_rng(n + 31 * d + K * L)
    X = rng.normal(size=(n, d)).astype(np.float32)
    Q = (X[rng.integers(0, n, size=m)] + 0.2 * rng.normal(size=(m, d))).astype(np.float32)
    if d == 784:
        X = synth.sparse_uniform(n, d, 11)
        Q = X[rng.integers(0, n, size=m)]
    announce(f"e2lsh table n={n} m={m} d={d} K={K} L={L}")
    _compare(stag, orc, X, Q, K, L, 900 + n)
