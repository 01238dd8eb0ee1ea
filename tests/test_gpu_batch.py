"""Batched path through the C ABI: every item of a batch of uneven sizes,
run eagerly, captured into a HIP graph and replayed, or autotuned, gives bit
for bit the oracle's outputs: its stream, its level-0 reconstruction and the
mesh of every isovalue (the oracle's marching cubes on the oracle's
reconstruction).  The single-field GPU calls give the same.  Tile shapes of
the level-0 kernels never change a result."""
import numpy as np
import pytest
import torch

import oracle
from paper_2408_05462_amd import api, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

# (shape, levels, block, relative error bound, number of isovalues)
ITEMS = [
    ((33, 40, 47), 3, 16, 1e-3, 3),
    ((64, 64, 64), 4, 32, 1e-3, 8),
    ((17, 23, 29), 2, 8, 1e-2, 1),
    ((65, 66, 67), 3, 32, 5e-4, 2),
    ((40, 37, 70), 3, 4, 1e-2, 4),
    ((96, 96, 96), 5, 64, 1e-3, 2),
]


def _fields():
    out = []
    for i, (shape, nL, B, rel, nk) in enumerate(ITEMS):
        n = max(shape)
        f = np.ascontiguousarray(inputs.grf(n, 0.25 * i)[: shape[0], : shape[1], : shape[2]])
        e = inputs.abs_error_bound(rel, f)
        isos = [float(v) for v in np.quantile(f, np.linspace(0.15, 0.85, nk)).astype(np.float32)]
        out.append((f, e, isos, nL, B))
    return out


@pytest.fixture(scope="module")
def data():
    """The expected outputs of every item, all from the oracle."""
    fields = _fields()
    xs = [torch.from_numpy(f).to(DEV) for f, *_ in fields]
    singles = []
    for f, e, isos, nL, B in fields:
        ref = oracle.compress(f, e, isos, levels=nL, block=B)
        y = oracle.decompress(ref["stream"], 0)
        meshes = [oracle.mc(y, k)[:2] for k in isos]
        singles.append((ref["stream"].tobytes(), y, meshes))
    return fields, xs, singles


def _batch(fields, xs):
    return api.Batch(xs, [e for _, e, *_ in fields], [isos for _, _, isos, *_ in fields],
                     [api.params(nL, B) for *_, nL, B in fields])


def _check(batch, singles, what):
    for i, (s_ref, y_ref, m_ref) in enumerate(singles):
        stream, r, y, meshes, st = batch.outputs(i)
        assert r["status"] == 0 and st == 0, (what, i)
        assert stream == s_ref, (what, i)
        assert np.array_equal(y.view(np.uint32), y_ref.view(np.uint32)), (what, i)
        for j, ((v, t), (vr, tr)) in enumerate(zip(meshes, m_ref)):
            assert np.array_equal(v.view(np.uint32), vr.view(np.uint32)), (what, i, j)
            assert np.array_equal(t, tr), (what, i, j)


def test_single_calls_match_the_oracle(data):
    fields, xs, singles = data
    for i, ((f, e, isos, nL, B), x, (s_ref, y_ref, m_ref)) in enumerate(zip(fields, xs, singles)):
        print("item", i, f.shape, flush=True)
        c = api.compress(x, e, isos, levels=nL, block=B)
        assert c.stream.cpu().numpy().tobytes() == s_ref, i
        y = api.reconstruct(c, 0)
        assert np.array_equal(y.cpu().numpy().view(np.uint32), y_ref.view(np.uint32)), i
        for j, k in enumerate(isos):
            v, t = api.extract(y, k)
            assert np.array_equal(v.cpu().numpy().view(np.uint32), m_ref[j][0].view(np.uint32)), (i, j)
            assert np.array_equal(t.cpu().numpy(), m_ref[j][1]), (i, j)


def test_batch_eager_matches_oracle(data):
    fields, xs, singles = data
    b = _batch(fields, xs)
    for r in b.recon:
        r.zero_()
    b.run()
    torch.cuda.synchronize()
    _check(b, singles, "eager")
    b.close()


def test_batch_graph_replays_match_oracle(data):
    fields, xs, singles = data
    b = _batch(fields, xs)
    b.capture()
    for rep in range(3):
        # eager work and synchronisation between replays; outputs cleared first
        for r in b.recon:
            r.fill_(float("nan"))
        for c in b.counts:
            c.zero_()
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        _check(b, singles, f"replay {rep}")
    b.close()


def test_batch_branch_counts_give_the_same_outputs(data):
    fields, xs, singles = data
    for br, ec, dc in [(1, 8, 16), (3, 2, 32), (len(ITEMS), 16, 8)]:
        b = _batch(fields, xs)
        b.set_config(br, ec, dc)
        b.capture()
        assert b.config()["branches"] == br
        for r in b.recon:
            r.fill_(float("nan"))
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        _check(b, singles, f"branches {br}, tiles {ec}/{dc}")
        b.close()


@pytest.mark.skip(reason="chr_batch_autotune is switched off: one GPU run aborted inside its replay-timed search "
                         "(SIGABRT, no fault message) and the cause is not yet known")
def test_batch_autotune_and_cache(data, tmp_path):
    fields, xs, singles = data
    cache = tmp_path / "tune.txt"
    b = _batch(fields, xs)
    b.autotune(cache)
    cfg = b.config()
    print("tuned", cfg, flush=True)
    assert cfg["last_ms"] > 0
    assert 1 <= cfg["branches"] <= len(ITEMS)
    b.replay()
    torch.cuda.synchronize()
    _check(b, singles, f"tuned {cfg}")
    lines = cache.read_text().split()
    assert len(lines) == 4 and [int(v) for v in lines[1:]] == [cfg["branches"], cfg["enc_cpw"], cfg["dec_cpw"]]
    # a second batch of the same shapes takes its configuration from the cache
    b2 = _batch(fields, xs)
    b2.autotune(cache)
    assert {k: v for k, v in b2.config().items() if k != "last_ms"} == \
        {k: v for k, v in cfg.items() if k != "last_ms"}
    assert len(cache.read_text().splitlines()) == 1
    b2.replay()
    torch.cuda.synchronize()
    _check(b2, singles, "cached")
    b.close()
    b2.close()


def test_batch_tune_picks_a_configuration_and_keeps_outputs(data, tmp_path):
    """The eager-timed search (brick size, branches, tiles) ends with a
    captured graph whose replays give the oracle's outputs for the chosen
    brick size (the oracle's stream at that size; reconstructions and meshes
    do not depend on it); a second batch takes the configuration from the
    cache file."""
    fields, xs, singles = data
    cache = tmp_path / "tune.txt"
    b = _batch(fields, xs)
    B = b.tune(cache)
    cfg = b.config()
    print("tuned", B, cfg, flush=True)
    assert B in (0, 32, 64, 128) and 1 <= cfg["branches"] <= len(ITEMS) and cfg["last_ms"] > 0
    refs = singles
    if B:
        refs = []
        for (f, e, isos, nL, _), (s_ref, y_ref, m_ref) in zip(fields, singles):
            refs.append((oracle.compress(f, e, isos, levels=nL, block=B)["stream"].tobytes(), y_ref, m_ref))
    for r in b.recon:
        r.fill_(float("nan"))
    torch.cuda.synchronize()
    b.replay()
    torch.cuda.synchronize()
    _check(b, refs, f"tuned {B} {cfg}")
    line = cache.read_text().split()
    assert len(line) == 5 and [int(v) for v in line[1:]] == [cfg["branches"], B, cfg["enc_cpw"], cfg["dec_cpw"]]
    b2 = _batch(fields, xs)
    assert b2.tune(cache) == B
    assert len(cache.read_text().splitlines()) == 1
    for r in b2.recon:
        r.fill_(float("nan"))
    torch.cuda.synchronize()
    b2.replay()
    torch.cuda.synchronize()
    _check(b2, refs, "cached")
    b.close()
    b2.close()


def test_tiles_do_not_change_results(data):
    fields, xs, singles = data
    f, e, isos, nL, B = fields[5]
    x = xs[5]
    s_ref, y_ref, _ = singles[5]
    try:
        for ec in (1, 2, 4, 8, 16):
            api.chr_set_tiles(ec, 16)
            c = api.compress(x, e, isos, levels=nL, block=B)
            assert c.stream.cpu().numpy().tobytes() == s_ref, ec
        c = api.compress(x, e, isos, levels=nL, block=B)
        for dc in (8, 16, 32, 64):
            api.chr_set_tiles(4, dc)
            y = api.reconstruct(c, 0).cpu().numpy()
            assert np.array_equal(y.view(np.uint32), y_ref.view(np.uint32)), dc
    finally:
        api.chr_set_tiles(8, 16)
