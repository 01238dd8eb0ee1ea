"""chr_reconstruct_static (no workspace, no allocation) against
chr_reconstruct, through the C ABI: bit for bit on two calls in a row, the
second on a smaller stream, at level 0 and a coarser level; a level whose
coarser grids exceed the static array is refused before any launch."""
import numpy as np
import pytest
import torch

from paper_2408_05462_amd import _lib as L
from paper_2408_05462_amd import api, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _stream(shape, nL, B, seed):
    n = max(shape)
    f = np.ascontiguousarray(inputs.grf(n, 0.1 * seed)[: shape[0], : shape[1], : shape[2]])
    e = inputs.abs_error_bound(1e-3, f)
    isos = [float(v) for v in np.quantile(f, [0.3, 0.7]).astype(np.float32)]
    return api.compress(torch.from_numpy(f).to(DEV), e, isos, levels=nL, block=B)


def _plain(c, level):
    shape = api.level_shape(c.info, level)
    out = torch.empty(shape, dtype=torch.float32, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    ws = torch.empty(max(api.chr_reconstruct_workspace(c.info, level), 256), dtype=torch.uint8, device=DEV)
    api.chr_reconstruct(c.info, c.stream, level, api.stream_bound(c.info), out, st, ws)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return out


def _static(c, level):
    shape = api.level_shape(c.info, level)
    out = torch.full(shape, float("nan"), dtype=torch.float32, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    api.chr_reconstruct_static(c.info, c.stream, level, api.stream_bound(c.info), out, st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return out


def test_static_matches_workspace_call_twice_in_a_row():
    big = _stream((160, 150, 170), 5, 64, 1)
    small = _stream((40, 33, 70), 3, 16, 2)
    for level in (0, 1):
        for c, what in ((big, "big"), (small, "small")):
            print("static reconstruction", what, level, flush=True)
            ref = _plain(c, level)
            got = _static(c, level)
            assert torch.equal(got.view(torch.int32), ref.view(torch.int32)), (what, level)


def test_static_refuses_levels_beyond_its_array():
    # 1024 x 1024 x 200 points: level 0 needs ~120 MB of coarser grids
    shape = (200, 1024, 1024)
    x = torch.zeros(shape, dtype=torch.float32, device=DEV)
    c = api.compress(x, 1e-3, [], levels=3, block=64)
    out = torch.empty(shape, dtype=torch.float32, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    assert api.chr_reconstruct_workspace(c.info, 0) > (96 << 20)
    with pytest.raises(L.ChrError) as ei:
        api.chr_reconstruct_static(c.info, c.stream, 0, 1e-3, out, st)
    assert ei.value.code == L.CHR_E_NOMEM
    # a coarser level of the same stream fits
    ref = _plain(c, 1)
    got = _static(c, 1)
    assert torch.equal(got.view(torch.int32), ref.view(torch.int32))
