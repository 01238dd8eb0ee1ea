"""GPU parity of multi-tier progressive accuracy against the oracle, through
the C ABI: the container byte for byte, the reconstruction at every tier's
bound bit for bit (from the GPU's container and from the oracle's), the
accuracy selection, and the capacity report.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2408_05462_amd import api, inputs
from paper_2408_05462_amd import _lib as L

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

# (shape, levels, block, relative tier bounds, isovalues)
CASES = [
    ((30, 31, 29), 3, 8, [1e-2, 1e-3, 1e-4, 0.0], [0.5, 1.0]),
    ((24, 24, 24), 4, 8, [5e-2, 5e-3], [-0.3]),
    ((17, 30, 9), 2, 4, [1e-2, 2e-3, 4e-4], [0.0, 0.7, 1.4]),
    ((65, 66, 67), 4, 16, [1e-2, 1e-3, 1e-4], [0.2]),
    ((40, 37, 70), 5, 16, [3e-2, 3e-3, 3e-4, 3e-5], [-1.0, 0.0, 1.0, 1.5]),
    ((1, 30, 31), 2, 2, [1e-2, 1e-3], []),                   # a one-point axis, no candidates
    ((9, 1, 5), 1, 1, [1e-1, 0.0], [0.2]),                    # one level, lossless last tier
]
IDS = [f"{'x'.join(map(str, c[0]))}-L{c[1]}-T{len(c[3])}" for c in CASES]


def _setup(case):
    shape, nL, B, rel, isos = case
    n = max(shape)
    f = np.ascontiguousarray(inputs.grf(n, 0.7)[: shape[0], : shape[1], : shape[2]])
    r = float(f.max() - f.min())
    return f, [v * r for v in rel], [float(np.float32(k)) for k in isos], nL, B


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_tier_container_bitexact(case):
    f, bounds, isos, nL, B = _setup(case)
    print("tiers compress", case[:3], flush=True)
    want = oracle.tiers_compress(f, bounds, isos, levels=nL, block=B)
    x = torch.from_numpy(f).to(DEV)
    c, h = api.tiers_compress(x, bounds, isos, levels=nL, block=B)
    got = c.cpu().numpy()
    assert got.size == want.size
    assert np.array_equal(got, want)
    assert h.n_tiers == len(bounds) and h.total_bytes == want.size


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_tier_reconstruct_every_bound(case):
    f, bounds, isos, nL, B = _setup(case)
    print("tiers reconstruct", case[:3], flush=True)
    want = oracle.tiers_compress(f, bounds, isos, levels=nL, block=B)
    cdev = torch.from_numpy(want).to(DEV)      # the oracle's container: independent of the GPU encoder
    h = api.chr_tiers_header(want[:640])
    for t, e in enumerate(bounds):
        y_ref, used_ref = oracle.tiers_decompress(want, e)
        y, used = api.tiers_reconstruct(cdev, h, e)
        assert used == used_ref == t
        assert np.array_equal(y.cpu().numpy().view(np.uint32), y_ref.view(np.uint32)), t
    with pytest.raises(L.ChrError):
        api.tiers_reconstruct(cdev, h, bounds[-1] * 0.5 if bounds[-1] > 0 else -1.0)
    if bounds[-1] == 0.0:
        y, _ = api.tiers_reconstruct(cdev, h, 0.0)
        assert np.array_equal(y.cpu().numpy().view(np.uint32), f.view(np.uint32))


def test_tier_capacity_reported_and_nothing_written_past_it():
    f, bounds, isos, nL, B = _setup(CASES[0])
    want = oracle.tiers_compress(f, bounds, isos, levels=nL, block=B)
    x = torch.from_numpy(f).to(DEV)
    p = api.params(nL, B)
    out = torch.full((want.size + 64,), 0xA5, dtype=torch.uint8, device=DEV)
    ws = torch.empty(api.chr_tiers_workspace(f.shape, p), dtype=torch.uint8, device=DEV)
    res = torch.zeros(2, dtype=torch.int64, device=DEV)
    cap = want.size - 8
    api.chr_tiers_compress(x, bounds, isos, p, out[:cap], res, ws)
    torch.cuda.synchronize()
    assert res.cpu().tolist() == [want.size, L.CHR_E_CAPACITY]
    assert bool((out[cap:] == 0xA5).all())
    api.chr_tiers_compress(x, bounds, isos, p, out[: want.size], res, ws)
    torch.cuda.synchronize()
    assert res.cpu().tolist() == [want.size, 0]
    assert np.array_equal(out[: want.size].cpu().numpy(), want)
