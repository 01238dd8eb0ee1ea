"""The paper's error translation (Sec. II.B) on the GPU against the oracle:
the bound (min or n-th smallest of D) bit for bit, and |D| exactly."""
import numpy as np
import pytest
import torch

import oracle
from paper_2408_05462_amd import api, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _fields():
    rng = np.random.default_rng(11)
    out = [
        ("normal", rng.standard_normal((17, 23, 29)).astype(np.float32), [-0.3, 0.4]),
        ("grf", np.ascontiguousarray(inputs.grf(70, 0.7)[:40, :37, :70]), [-1.0, 0.0, 0.5]),
        ("flat-axis", rng.standard_normal((1, 30, 31)).astype(np.float32), [0.1]),
        ("line", rng.standard_normal((9, 1, 1)).astype(np.float32), [0.0, 0.0]),  # duplicates count twice
        ("ragged", rng.standard_normal((65, 3, 67)).astype(np.float32), [0.2, -0.2, 1.5, -2.5]),
    ]
    g = inputs.gaussians(64)
    out.append(("gaussians64", g, [0.3]))
    return out


@pytest.mark.parametrize("case", _fields(), ids=lambda c: c[0])
def test_topology_bound_matches_oracle(case):
    name, f, isos = case
    print("case", name, f.shape, isos, flush=True)
    x = torch.from_numpy(f).to(DEV)
    r1, m = oracle.topology_error_bound(f, isos, nth=1)
    g1, gm = api.topology_error_bound(x, isos, nth=1)
    assert gm == m
    assert np.float64(g1).tobytes() == np.float64(r1).tobytes()
    if m == 0:
        assert np.isinf(g1)
        return
    for nth in sorted({0, 2, 3, 7, m // 3, m // 2, m - 1, m, m + 5}):
        r, _ = oracle.topology_error_bound(f, isos, nth=nth)
        g, gm2 = api.topology_error_bound(x, isos, nth=nth)
        assert gm2 == m
        assert np.float64(g).tobytes() == np.float64(r).tobytes(), nth


def test_topology_bound_empty_and_far_isovalues():
    f = np.full((8, 9, 10), 2.0, np.float32)
    x = torch.from_numpy(f).to(DEV)
    for nth in (1, 4):
        g, m = api.topology_error_bound(x, [2.0, 5.0], nth=nth)  # equal values never enclose k strictly
        assert m == 0 and np.isinf(g)
    g, m = api.topology_error_bound(x, [], nth=1)
    assert m == 0 and np.isinf(g)


def test_topology_bound_keeps_crossings_when_used_as_error_bound():
    """Compressing with an error bound below min(D) keeps every crossing edge
    crossing (Sec. II.B); the oracle checks the reconstruction's crossings."""
    f = inputs.gaussians(48)
    k = 0.3
    x = torch.from_numpy(f).to(DEV)
    b, m = api.topology_error_bound(x, [k], nth=1)
    assert m > 0
    e = float(np.nextafter(b, 0.0))  # strictly below min(D)
    c = api.compress(x, e, [], levels=3, block=16)  # no candidates: the bound alone must keep the crossings
    y = api.reconstruct(c, 0).cpu().numpy().astype(np.float64)
    fd = f.astype(np.float64)
    for a in range(3):
        s0 = np.take(fd, range(f.shape[a] - 1), axis=a)
        s1 = np.take(fd, range(1, f.shape[a]), axis=a)
        t0 = np.take(y, range(f.shape[a] - 1), axis=a)
        t1 = np.take(y, range(1, f.shape[a]), axis=a)
        cross = (np.minimum(s0, s1) < k) & (k < np.maximum(s0, s1))
        assert np.all(((np.minimum(t0, t1) < k) & (k < np.maximum(t0, t1)))[cross])
