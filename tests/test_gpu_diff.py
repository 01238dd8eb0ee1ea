"""GPU parity of differentiated error control (blocks with different error
bounds, Sec. II.A) against the oracle, through the C ABI.

Streams, codes and flags are compared byte for byte with the oracle's; the
reconstruction at every level bit for bit; the GPU decodes the oracle's own
streams; the meshes of the candidate isovalues equal those of a stream with
the near bound everywhere; restricted reconstruction and the batched path
give the single calls' results.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2408_05462_amd import api, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

# (shape, levels, block, relative near bound, relative far bound, isovalues)
CASES = [
    ((40, 37, 45), 3, 8, 1e-3, 3e-2, [2.0]),
    ((33, 33, 33), 4, 8, 1e-3, 3e-2, [-2.2, 2.4]),
    ((17, 30, 9), 3, 4, 1e-3, 2e-2, [1.0, 1.5, 2.0]),
    ((65, 66, 67), 5, 16, 5e-4, 1e-2, [2.1]),
    ((20, 21, 22), 1, 4, 1e-3, 5e-2, [1.5]),
    ((70, 65, 129), 5, 16, 1e-4, 1e-2, list(np.linspace(2.2, 3.0, 16))),
    ((24, 24, 24), 3, 8, 0.0, 1e-2, [2.0]),      # near blocks lossless
    ((20, 21, 22), 3, 8, 1e-3, 2e-2, []),        # no candidates: the far bound everywhere
]
IDS = [f"{'x'.join(map(str, c[0]))}-L{c[1]}-B{c[2]}-K{len(c[5])}" for c in CASES]


def _setup(case):
    shape, nL, B, rn, rf, isos = case
    n = max(shape)
    f = np.ascontiguousarray(inputs.grf(n, 0.5)[: shape[0], : shape[1], : shape[2]])
    r = float(f.max() - f.min())
    isos = [float(np.float32(k)) for k in isos]
    return f, rn * r, rf * r, isos, nL, B


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_diff_compress_bitexact(case):
    f, e, ef, isos, nL, B = _setup(case)
    print("diff compress", case[:3], flush=True)
    ref = oracle.compress(f, e, isos, levels=nL, block=B, error_bound_far=ef)
    x = torch.from_numpy(f).to(DEV)
    codes = torch.zeros(f.shape, dtype=torch.int32, device=DEV)
    flags = torch.zeros(f.shape, dtype=torch.uint8, device=DEV)
    c = api.compress(x, e, isos, levels=nL, block=B, codes=codes, flags=flags, error_bound_far=ef)
    assert np.array_equal(codes.cpu().numpy(), ref["q"])
    assert np.array_equal(flags.cpu().numpy(), ref["flags"])
    assert np.array_equal(c.stream.cpu().numpy(), ref["stream"])
    assert c.info.flags & 2 and c.info.error_bound_far == ef
    # without the per-point outputs (the specialized kernels' other variant)
    c2 = api.compress(x, e, isos, levels=nL, block=B, error_bound_far=ef)
    assert np.array_equal(c2.stream.cpu().numpy(), ref["stream"])


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_diff_reconstruct_bitexact_every_level(case):
    f, e, ef, isos, nL, B = _setup(case)
    print("diff reconstruct", case[:3], flush=True)
    ref = oracle.compress(f, e, isos, levels=nL, block=B, error_bound_far=ef)
    s_dev = torch.from_numpy(ref["stream"]).to(DEV)
    oc = api.Compressed(stream=s_dev, info=api.chr_stream_info(bytes(ref["stream"])), header=b"", result={})
    for l in range(nL):
        y = api.reconstruct(oc, l).cpu().numpy()
        s = slice(None, None, 1 << l)
        assert np.array_equal(y.view(np.uint32), ref["xr"][s, s, s].view(np.uint32)), l
    # a request below the far bound is refused; the far bound is accepted
    if ef > e:
        with pytest.raises(api.L.ChrError):
            api.reconstruct(oc, 0, error_bound=0.5 * (e + ef))


@pytest.mark.parametrize("case", CASES[:4] + CASES[5:6], ids=IDS[:4] + IDS[5:6])
def test_diff_candidate_meshes_equal_uniform_and_restricted(case):
    f, e, ef, isos, nL, B = _setup(case)
    print("diff meshes", case[:3], flush=True)
    x = torch.from_numpy(f).to(DEV)
    cd = api.compress(x, e, isos, levels=nL, block=B, error_bound_far=ef)
    cu = api.compress(x, e, isos, levels=nL, block=B)
    assert cd.stream.numel() < cu.stream.numel()
    yd, yu = api.reconstruct(cd, 0), api.reconstruct(cu, 0)
    for k in isos:
        vd, td = api.extract(yd, k)
        vu, tu = api.extract(yu, k)
        assert torch.equal(td, tu)
        assert torch.equal(vd.view(torch.int32), vu.view(torch.int32))
        assert torch.equal(api.cases(yd, k), api.cases(x, k))
        # restricted reconstruction at the candidate: the same cases and mesh
        yr = api.reconstruct_range(cd, k, k)
        assert torch.equal(api.cases(yr, k), api.cases(x, k))
        vr, tr = api.extract(yr, k)
        assert torch.equal(tr, td) and torch.equal(vr.view(torch.int32), vd.view(torch.int32))


def test_diff_batch_matches_single_calls():
    items = [CASES[0], CASES[1], CASES[3]]
    setups = [_setup(c) for c in items]
    xs = [torch.from_numpy(f).to(DEV) for f, *_ in setups]
    singles = []
    for (f, e, ef, isos, nL, B), x in zip(setups, xs):
        c = api.compress(x, e, isos, levels=nL, block=B, error_bound_far=ef)
        singles.append((c.stream.cpu().numpy().tobytes(), api.reconstruct(c, 0).cpu().numpy()))
    b = api.Batch(xs, [s[1] for s in setups], [s[3] for s in setups],
                  [api.params(s[4], s[5], error_bound_far=s[2]) for s in setups])
    b.run()
    torch.cuda.synchronize()
    for i, (s_ref, y_ref) in enumerate(singles):
        stream, r, y, meshes, st = b.outputs(i)
        assert r["status"] == 0 and st == 0, i
        assert stream == s_ref, i
        assert np.array_equal(y.view(np.uint32), y_ref.view(np.uint32)), i
    b.close()


def test_diff_restricted_reconstruction_off_the_candidates():
    # a range holding no candidate decodes near and far blocks side by side:
    # their shared points carry one value, so the cases and mesh at any
    # isovalue of the range equal the full reconstruction's
    f, e, ef, isos, nL, B = _setup(CASES[0])
    x = torch.from_numpy(f).to(DEV)
    cd = api.compress(x, e, isos, levels=nL, block=B, error_bound_far=ef)
    y = api.reconstruct(cd, 0)
    for k in (0.5, 1.2):
        yr = api.reconstruct_range(cd, k, k)
        assert torch.equal(api.cases(yr, k), api.cases(y, k))
        v, t = api.extract(y, k)
        vr, tr = api.extract(yr, k)
        assert torch.equal(tr, t) and torch.equal(vr.view(torch.int32), v.view(torch.int32))
