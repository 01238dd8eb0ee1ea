"""Restricted reconstruction (chr_reconstruct_range): blocks that cannot
hold the isosurface of any isovalue in [kmin, kmax] are skipped, and for
every such isovalue the marching-cubes cases and meshes are bit for bit those
of the full reconstruction; reconstructed blocks hold the full
reconstruction's values."""
import numpy as np
import pytest
import torch

import oracle
from paper_2408_05462_amd import api, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _fields():
    g = inputs.gaussians(64)
    z, y, x = np.meshgrid(*[np.linspace(0, 3, n) for n in (70, 65, 129)], indexing="ij")
    smooth = (np.sin(x + 0.3 * y) * np.cos(y - z)).astype(np.float32)
    return [("gaussians64", g, 3, 16, [0.3, 0.6]),
            ("smooth", smooth, 4, 16, [0.0, 0.5]),
            ("grf", np.ascontiguousarray(inputs.grf(80, 0.2)[:70, :80, :75]), 3, 32, [-0.5, 0.5])]


def _needed(stream_bytes, kmin, kmax):
    mins, maxs = oracle.block_index(stream_bytes)
    return (mins < maxs) & (mins < kmax) & (kmin <= maxs)


@pytest.mark.parametrize("case", _fields(), ids=lambda c: c[0])
def test_range_reconstruction_keeps_meshes(case):
    name, f, nL, B, isos = case
    x = torch.from_numpy(f).to(DEV)
    e = inputs.abs_error_bound(1e-3, f)
    c = api.compress(x, e, isos, levels=nL, block=B)
    full = api.reconstruct(c, 0)
    lo, hi = float(f.min()), float(f.max())
    ranges = [(isos[0], isos[0]), (isos[0], isos[1]), (lo + 0.9 * (hi - lo), hi), (lo, lo + 0.05 * (hi - lo))]
    host = c.stream.cpu().numpy()
    pruned_any = False
    for kmin, kmax in ranges:
        kmin, kmax = float(np.float32(kmin)), float(np.float32(kmax))
        need = _needed(host, kmin, kmax)
        pruned_any |= not need.all()
        print(name, kmin, kmax, "blocks needed", int(need.sum()), "of", need.size, flush=True)
        y = api.reconstruct_range(c, kmin, kmax, 0)
        for k in sorted({kmin, kmax, float(np.float32(0.5 * (kmin + kmax)))}):
            assert torch.equal(api.cases(y, k), api.cases(full, k)), (kmin, kmax, k)
            v, t = api.extract(y, k)
            vf, tf = api.extract(full, k)
            assert torch.equal(v.view(torch.int32), vf.view(torch.int32)) and torch.equal(t, tf), (kmin, kmax, k)
        # reconstructed blocks hold the full reconstruction's values
        yh, fh = y.cpu().numpy(), full.cpu().numpy()
        nb = [(n - 2) // B + 1 if n > 1 else 1 for n in f.shape]
        for b in np.flatnonzero(need.reshape(-1)):
            bz, by, bx = np.unravel_index(b, nb)
            sl = tuple(slice(i * B, min(i * B + B, n - 1) + 1) for i, n in zip((bz, by, bx), f.shape))
            assert np.array_equal(yh[sl].view(np.uint32), fh[sl].view(np.uint32)), (kmin, kmax, b)
    assert pruned_any


def test_range_reconstruction_at_a_coarser_level():
    f = inputs.gaussians(64)
    x = torch.from_numpy(f).to(DEV)
    c = api.compress(x, inputs.abs_error_bound(1e-3, f), [0.3], levels=3, block=16)
    for level in (1, 2):
        full = api.reconstruct(c, level)
        y = api.reconstruct_range(c, 0.3, 0.45, level)
        for k in (0.3, 0.4, 0.45):
            kk = float(np.float32(k))
            v, t = api.extract(y, kk, spacing=float(1 << level))
            vf, tf = api.extract(full, kk, spacing=float(1 << level))
            assert torch.equal(v.view(torch.int32), vf.view(torch.int32)) and torch.equal(t, tf), (level, k)


def test_range_reconstruction_rejects_bad_ranges():
    f = inputs.gaussians(32)
    x = torch.from_numpy(f).to(DEV)
    c = api.compress(x, 1e-3, [0.3], levels=3, block=16)
    for kmin, kmax in [(0.5, 0.4), (float("nan"), 0.4), (0.1, float("inf"))]:
        with pytest.raises(api.L.ChrError):
            api.reconstruct_range(c, kmin, kmax, 0)
