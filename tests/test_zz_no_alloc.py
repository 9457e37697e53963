"""The no-allocation energy entry point (nnqs_energy_noalloc) against the
table-scratch one (nnqs_energy) it varies: two calls in a row, the second
with a smaller input, both through the C ABI; results must be bit-identical
(same kernels, same reduction order)."""
import numpy as np
import pytest
import torch

from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_16705_amd as nn
    return nn


def _inputs(n, seed):
    rng = np.random.default_rng([16705, 92, seed])
    el = np.stack([rng.normal(-130.0, 3.0, size=n), rng.normal(0.0, 0.5, size=n)], axis=1)
    cnt = np.maximum(1, rng.poisson(20.0, size=n)).astype(np.uint32)
    return dev(cnt, torch.int32), dev(el)


def test_noalloc_energy_matches_table_energy_twice(nn):
    print("[case] energy_noalloc n=300001 then n=4097", flush=True)
    S = nn.System(8, 2, 2, np.eye(4), np.zeros((4, 4, 4, 4)))
    T = nn.Table(S, capacity=4)
    for n, seed in ((300001, 1), (4097, 2)):
        cnt, el = _inputs(n, seed)
        a = nn.energy(T, cnt, el)
        b = torch.full((4,), np.nan, dtype=torch.float64, device="cuda")
        nn.energy_noalloc(cnt, el, out=b)
        torch.cuda.synchronize()
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.all(np.isfinite(b))
        assert (a == b).all(), (n, a, b)


def test_noalloc_energy_rejects_bad_sizes(nn):
    cnt, el = _inputs(16, 3)
    out = torch.full((4,), 7.0, dtype=torch.float64, device="cuda")
    from paper_2306_16705_amd import _lib as L
    lib = L.load()
    r = lib.nnqs_energy_noalloc(cnt.data_ptr(), el.data_ptr(), 0, out.data_ptr(), None)
    assert r == -1
    r = lib.nnqs_energy_noalloc(cnt.data_ptr(), el.data_ptr(), (1 << 31), out.data_ptr(), None)
    assert r == -4 and b"no-allocation limit" in lib.nnqs_last_error()
    torch.cuda.synchronize()
    assert (out == 7.0).all()
