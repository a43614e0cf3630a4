"""The random-gather calibration kernel (grest_calib_gather) computes what its header
states: the sum, for every row, of the rows of Z picked by the splitmix64 finaliser of the
indices of the row's entries.  The benchmark times it as the ceiling of the sparse product."""
import numpy as np
import pytest
import torch

from paper_2603_19439_amd import grest as G

pytestmark = pytest.mark.gpu


def splitmix_finaliser(x):
    x = x.astype(np.uint64)
    with np.errstate(over="ignore"):
        x ^= x >> np.uint64(30)
        x *= np.uint64(0xBF58476D1CE4E5B9)
        x ^= x >> np.uint64(27)
        x *= np.uint64(0x94D049BB133111EB)
        x ^= x >> np.uint64(31)
    return (x & np.uint64(0xFFFFFFFF)).astype(np.uint64)


@pytest.mark.parametrize("n,m,w,ld,seed", [(1000, 20_017, 64, 96, 3), (777, 5_000, 196, 196, 11), (5, 0, 4, 4, 1)])
def test_calib_gather_matches_its_definition(n, m, w, ld, seed):
    rng = np.random.default_rng(seed)
    Zh = rng.standard_normal((n, ld)).astype(np.float32)
    Z = torch.from_numpy(Zh).cuda()
    Y = torch.full((n, ld), 7.0, device="cuda")
    rph = np.arange(n + 1, dtype=np.int64) * m // n
    rph[1:-1] += rng.integers(-3, 4, n - 1) if m >= 8 * n else 0  # uneven rows, still nondecreasing
    rph = np.maximum.accumulate(np.clip(rph, 0, m))
    G.calib_gather(torch.from_numpy(rph).cuda(), Z, w, Y, seed=seed)
    torch.cuda.synchronize()
    Yh = Y.cpu().numpy()
    cols = (splitmix_finaliser(np.uint64(seed) + np.arange(m, dtype=np.uint64)) % np.uint64(n)).astype(np.int64)
    ref = np.zeros((n, w))
    for r in range(n):
        b, e = rph[r], rph[r + 1]
        ref[r] = Zh[cols[b:e], :w].astype(np.float64).sum(axis=0)
    assert np.abs(Yh[:, :w] - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())
    assert np.all(Yh[:, w:] == 7.0)  # columns beyond w untouched
