"""chi2_noalloc (the chi2 entry point that allocates nothing: its scratch is a
static device array of the library) against chi2 with a caller workspace,
called through the C ABI: two calls in a row, the second on a smaller input,
in single and double precision.  Bar: relative 1e-12 (both sum the same terms
in FP64, over a different split of the orbits)."""
import numpy as np
import pytest

from tests.gpu_common import lib

pytestmark = pytest.mark.gpu


def _problem(n, nc, dtype, seed, dev):
    import torch
    rng = np.random.default_rng(seed)
    A = rng.uniform(0, 1, size=(n, nc)) * (rng.random((n, nc)) < 0.1)
    w = rng.exponential(1.0, n) * (rng.random(n) < 0.3)
    d = A.T @ w * (1 + 0.05 * rng.normal(size=nc)) + 1e-3
    sig = 0.03 * np.maximum(d, 1e-3)
    td = torch.float32 if dtype == "f32" else torch.float64
    return (torch.from_numpy(A).to(dev, td), torch.from_numpy(w).to(dev), torch.from_numpy(d).to(dev),
            torch.from_numpy(sig).to(dev))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_chi2_noalloc_matches_chi2(gpu, dtype):
    import torch
    P = lib()
    assert P.chi2_noalloc_max_con() == 65536
    for k, (n, nc, cb, ce) in enumerate([(3000, 20000, 1500, 20000), (700, 1750, 1000, 1750)]):
        A, w, d, s = _problem(n, nc, dtype, seed=10 + k, dev=gpu)
        ws = torch.empty(P.chi2_workspace_bytes(nc), dtype=torch.uint8, device=gpu)
        ref = P.chi2(A, w, d, s, cb, ce, ws)
        got = P.chi2_noalloc(A, w, d, s, cb, ce)
        assert got == pytest.approx(ref, rel=1e-12), (k, got, ref)
        assert got > 0
        whole = P.chi2_noalloc(A, w, d, s, 0, nc)
        assert whole == pytest.approx(P.chi2(A, w, d, s, 0, nc, ws), rel=1e-12)


def test_chi2_noalloc_rejects_beyond_its_limit(gpu):
    import torch
    P = lib()
    n, nc = 4, 65537
    A = torch.zeros((n, nc), dtype=torch.float32, device=gpu)
    w = torch.zeros(n, dtype=torch.float64, device=gpu)
    d = torch.zeros(nc, dtype=torch.float64, device=gpu)
    with pytest.raises(P.SchwError) as e:
        P.chi2_noalloc(A, w, d, d + 1, 0, nc)
    assert "exceeds the static scratch limit" in str(e.value)
