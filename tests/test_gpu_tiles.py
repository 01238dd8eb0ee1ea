"""The level-0 kernels that work by pairs of z-planes (64-cell blocks) against
the oracle, through the C ABI: stream bytes identical to the oracle's and to
the one-wave-per-chunk kernels' on fields whose blocks are cut short on every
axis (1, 2, ... points left), one block, one plane, a lossless stream (every
point stored exactly), forced outliers (small qmax) and 16 candidates; the
level-0 reconstruction by either decoder is the oracle's bit for bit, also
from the oracle's own stream; a reconstruction restricted to an isovalue
range is the same by either decoder and keeps every cell's case.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2408_05462_amd import api, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _field(kind, shape, seed):
    rng = np.random.default_rng(seed)
    if kind == "normal":
        return rng.standard_normal(shape).astype(np.float32)
    if kind == "smooth":
        z, y, x = np.meshgrid(*[np.linspace(0, 3, n) for n in shape], indexing="ij")
        return (np.sin(x + 0.3 * y) * np.cos(y - z) + 0.01 * rng.standard_normal(shape)).astype(np.float32)
    if kind == "grf":
        n = max(shape)
        return np.ascontiguousarray(inputs.grf(n, 0.5)[: shape[0], : shape[1], : shape[2]])
    raise KeyError(kind)


CASES = [
    # (kind, shape, levels, relative error bound, number of isovalues, qmax)
    ("grf", (65, 65, 65), 2, 1e-3, 2, 32767),        # one whole block
    ("normal", (129, 130, 131), 3, 3e-2, 2, 32767),  # last blocks of 0, 1 and 2 cells
    ("smooth", (97, 64, 200), 4, 1e-3, 3, 32767),    # 33-, 64- and 8-point last blocks
    ("grf", (66, 127, 65), 6, 1e-3, 16, 32767),      # 16 candidates, 6 levels
    ("normal", (5, 70, 300), 2, 1e-2, 1, 32767),     # a thin slab
    ("normal", (65, 66, 67), 3, 0.0, 1, 32767),      # lossless: every level-0 point exact
    ("normal", (70, 66, 68), 3, 2e-3, 2, 4),         # most points outliers
    ("smooth", (2, 3, 2), 2, 1e-2, 1, 32767),        # one cell along z and x
    ("smooth", (1, 30, 131), 2, 1e-2, 1, 32767),     # one plane
    ("grf", (130, 129, 257), 3, 1e-3, 2, 32767),     # several blocks on every axis
]


def _ids(c):
    return f"{c[0]}-{'x'.join(map(str, c[1]))}-L{c[2]}-q{c[5]}"


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_plane_pair_kernels_match_oracle(case):
    kind, shape, nL, rel, nk, qmax = case
    print("case", case, flush=True)
    f = _field(kind, shape, 7)
    e = inputs.abs_error_bound(rel, f)
    isos = list(np.quantile(f, np.linspace(0.2, 0.8, nk)).astype(np.float32)) if nk else []
    ref = oracle.compress(f, e, isos, levels=nL, block=64, qmax=qmax)
    x = torch.from_numpy(f).to(DEV)
    try:
        api.chr_set_level0_tiles(True)
        ct = api.compress(x, e, isos, levels=nL, block=64, qmax=qmax)
        api.chr_set_level0_tiles(False)
        cc = api.compress(x, e, isos, levels=nL, block=64, qmax=qmax)
    finally:
        api.chr_set_level0_tiles(True)
    st, sc = ct.stream.cpu().numpy(), cc.stream.cpu().numpy()
    assert st.size == ref["stream"].size and np.array_equal(st, ref["stream"])
    assert sc.size == ref["stream"].size and np.array_equal(sc, ref["stream"])
    assert ct.result == cc.result
    assert ct.result["n_outlier"] == int((ref["flags"] & 1).sum())
    assert ct.result["n_corrected"] == int((ref["flags"] >> 1).sum())
    oc = api.Compressed(stream=torch.from_numpy(ref["stream"]).to(DEV),
                        info=api.chr_stream_info(bytes(ref["stream"])), header=b"", result={})
    try:
        for on in (True, False):
            api.chr_set_level0_tiles(on)
            for c in (ct, oc):
                y = api.reconstruct(c, 0).cpu().numpy()
                assert np.array_equal(y.view(np.uint32), ref["xr"].view(np.uint32)), on
        if isos:
            k = float(isos[0])
            rt = []
            for on in (True, False):
                api.chr_set_level0_tiles(on)
                rt.append(api.reconstruct_range(ct, k, k))
            assert torch.equal(rt[0].view(torch.int32), rt[1].view(torch.int32))
            assert torch.equal(api.cases(rt[0], k), api.cases(x, k))
    finally:
        api.chr_set_level0_tiles(True)
