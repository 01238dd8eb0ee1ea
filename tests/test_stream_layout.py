"""Pins the CHR stream's byte layout with a decoder of its own.

The reader below is written from the stream format alone (header fields at
fixed byte offsets, section table, block table, sections of 64-point chunks
with a tile table, width/exact header bytes, zigzag codes packed LSB first at
the chunk's width, exact masks and exact values) and shares nothing with the
oracle's reader: it finds every point of every section by walking the block's
closed extent itself, unpacks codes with numpy bit operations and recomputes
every checksum from MurmurHash3's 32-bit finalizer.  It then has to land on
the oracle's codes, exact flags and exact values at every grid point, on the
block minima and maxima of the oracle's reconstruction, and on the header's
counts, so that a section in the wrong order, a transposed block index, a
code bit out of place or a field at the wrong offset fails here.

The quantities being laid out are those of Sec. II.A (hierarchical levels,
error-bounded codes, points stored exactly) and Sec. II.B (corrected points);
the layout itself is this implementation's choice (the paper gives none).
"""
import struct

import numpy as np
import pytest

import oracle
from paper_2408_05462_amd import inputs

M32 = 0xFFFFFFFF


def _fmix32(h):
    """MurmurHash3's 32-bit finalizer, vectorised over uint64 holding u32s."""
    h = h ^ (h >> np.uint64(16))
    h = (h * np.uint64(0x85EBCA6B)) & np.uint64(M32)
    h = h ^ (h >> np.uint64(13))
    h = (h * np.uint64(0xC2B2AE35)) & np.uint64(M32)
    return h ^ (h >> np.uint64(16))


def _checksum(buf):
    n = len(buf) // 4
    w = np.frombuffer(bytes(buf[: 4 * n]), "<u4").astype(np.uint64)
    j = (np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B9)) & np.uint64(M32)
    return int(_fmix32(w ^ j).sum() & np.uint64(M32))


def _pad8(n):
    return (n + 7) & ~7


def _level(c, nL):
    """Level of each point of the coordinate triples c (shape [n, 3]): the
    fewest trailing zero bits among non-zero coordinates, at most nL-1."""
    lv = np.full(len(c), nL - 1, np.int64)
    for a in range(3):
        v = c[:, a]
        nz = v != 0
        tz = np.zeros(len(c), np.int64)
        lowbit = v[nz] & -v[nz]
        tz[nz] = np.log2(lowbit).astype(np.int64)
        lv = np.where(nz, np.minimum(lv, tz), lv)
    return lv


class Stream:
    def __init__(self, s):
        self.s = bytes(s)
        s = self.s
        u32 = lambda o: struct.unpack_from("<I", s, o)[0]
        u64 = lambda o: struct.unpack_from("<Q", s, o)[0]
        f32 = lambda o: struct.unpack_from("<f", s, o)[0]
        self.magic, self.version = u32(0), u32(4)
        self.dims = tuple(u64(8 + 8 * a) for a in range(3))
        self.nL, self.B, self.qmax, self.K = (u32(32 + 4 * a) for a in range(4))
        self.e = struct.unpack_from("<d", s, 48)[0]
        self.inv, self.step = f32(56), f32(60)
        self.iso = [f32(64 + 4 * j) for j in range(16)]
        self.vmin, self.vmax = f32(128), f32(132)
        self.nblocks = u64(136)
        self.nb = tuple(u32(144 + 4 * a) for a in range(3))
        self.flags = u32(156)
        self.total, self.nO, self.nC, self.payload = u64(160), u64(168), u64(176), u64(184)
        self.e_far = struct.unpack_from("<d", s, 192)[0]
        self.far_inv, self.far_step = f32(200), f32(204)
        self.tab_sum, self.hdr_sum = u32(248), u32(252)
        # flags bit 3: storage units are merged rectangles of blocks, listed
        # in a box table after the unit records
        self.merged = bool(self.flags & 8)
        self.merge = u32(208) if self.merged else 1
        self.mb = tuple(u32(212 + 4 * a) for a in range(3)) if self.merged else (1, 1, 1)
        self.u32, self.u64, self.f32 = u32, u64, f32

    def box(self, b):
        """First block and one past the last block of unit b (z, y, x)."""
        if self.merged:
            e = struct.unpack_from("<8I", self.s, 256 + 16 * self.nblocks * self.nL + 16 * self.nblocks + 32 * b)
            assert e[6] == 0 and e[7] == 0
            return e[:3], e[3:6]
        nby, nbx = self.nb[1], self.nb[2]
        bi = (b // (nby * nbx), (b // nbx) % nby, b % nbx)
        return bi, tuple(v + 1 for v in bi)

    def extent(self, b):
        b0, b1 = self.box(b)
        lo = [self.B * b0[a] for a in range(3)]
        hi = [min(self.B * b1[a], self.dims[a] - 1) for a in range(3)]
        return lo, hi

    def points(self, b, l):
        lo, hi = self.extent(b)
        h = 1 << l
        axes = [np.arange(lo[a], hi[a] + 1, dtype=np.int64) for a in range(3)]
        # a point of level l lies on the 2^l grid, and the block's origin is
        # a multiple of B, itself a multiple of 2^(nL-1)
        axes = [v[v % h == 0] for v in axes]
        g = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
        return g[_level(g, self.nL) == l]

    def section(self, b, l):
        ent = 256 + 16 * (b * self.nL + (self.nL - 1 - l))
        return self.u64(ent), self.u64(ent + 8)

    def decode_section(self, off, size, n):
        s, u32, u64 = self.s, self.u32, self.u64
        assert u32(off) == n
        W, NE, NX = u32(off + 4), u32(off + 8), u32(off + 12)
        nc = -(-n // 64)
        nt = -(-nc // 64)
        o_tile = off + 16
        o_hdr = o_tile + _pad8(12 * nt)
        o_pay = o_hdr + _pad8(nc)
        o_msk = o_pay + 8 * W
        o_ex = o_msk + 8 * NE
        assert size == o_ex + _pad8(4 * NX) - off
        hdr = np.frombuffer(s, np.uint8, nc, o_hdr)
        assert not (hdr & 0x60).any() and ((hdr & 31) <= 16).all()
        # padding bytes are zero
        assert not any(s[o_hdr + nc: o_pay]) and not any(s[o_tile + 12 * nt: o_hdr])
        assert not any(s[o_ex + 4 * NX: o_ex + _pad8(4 * NX)])
        width = (hdr & 31).astype(np.int64)
        has_e = (hdr >> 7).astype(np.int64)
        wbefore = np.concatenate([[0], np.cumsum(width)])
        ebefore = np.concatenate([[0], np.cumsum(has_e)])
        masks = np.frombuffer(s, "<u8", NE, o_msk)
        assert wbefore[-1] == W and ebefore[-1] == NE
        for t in range(nt):
            c = 64 * t
            got = struct.unpack_from("<III", s, o_tile + 12 * t)
            xb = sum(bin(int(m)).count("1") for m in masks[: ebefore[c]])
            assert got == (wbefore[c], ebefore[c], xb), (t, got)
        pay = np.frombuffer(s, np.uint8, 8 * W, o_pay)
        codes = np.zeros(64 * nc, np.int64)
        exact = np.zeros(64 * nc, bool)
        for c in range(nc):
            w = int(width[c])
            if w:
                bits = np.unpackbits(pay[8 * wbefore[c]: 8 * wbefore[c + 1]], bitorder="little")
                z = (bits.reshape(64, w).astype(np.int64) << np.arange(w)).sum(1)
                codes[64 * c: 64 * c + 64] = (z >> 1) ^ -(z & 1)
            if has_e[c]:
                m = int(masks[ebefore[c]])
                exact[64 * c: 64 * c + 64] = [(m >> i) & 1 for i in range(64)]
        assert not exact[n:].any() and not codes[n:].any()
        assert not codes[exact].any()
        assert int(exact.sum()) == NX
        vals = np.frombuffer(s, "<u4", NX, o_ex)
        # the width is the bit length of the OR of the chunk's zigzag codes
        zz = ((codes << 1) ^ (codes >> 63)).reshape(nc, 64)
        orv = np.bitwise_or.reduce(zz, axis=1)
        assert np.array_equal(width, np.array([int(v).bit_length() for v in orv]))
        return codes[:n], exact[:n], vals

    def decode(self):
        nz, ny, nx = self.dims
        q = np.full((nz, ny, nx), np.iinfo(np.int32).min, np.int64)
        ex = np.zeros((nz, ny, nx), np.int8) - 1
        xv = np.zeros((nz, ny, nx), np.uint32)
        seen = np.zeros((nz, ny, nx), np.int32)
        expect = self.payload
        for b in range(self.nblocks):
            first = expect
            for l in range(self.nL - 1, -1, -1):
                off, size = self.section(b, l)
                assert off == expect and off % 8 == 0, (b, l, off, expect)
                p = self.points(b, l)
                codes, exact, vals = self.decode_section(off, size, len(p))
                z, y, x = p[:, 0], p[:, 1], p[:, 2]
                first_time = seen[z, y, x] == 0
                # a point shared by neighbouring blocks is coded identically
                # in each of them
                assert np.array_equal(q[z, y, x][~first_time], codes[~first_time])
                assert np.array_equal(ex[z, y, x][~first_time], exact[~first_time])
                q[z, y, x] = codes
                ex[z, y, x] = exact
                xv[z[exact], y[exact], x[exact]] = vals
                seen[z, y, x] += 1
                expect = off + size
            rec = 256 + 16 * self.nblocks * self.nL + 16 * b
            assert self.u32(rec + 8) == _checksum(self.s[first:expect]), b
        assert expect == self.total == len(self.s)
        assert (seen > 0).all()
        return q, ex.astype(bool), xv


CASES = [
    # (field, shape, levels, block, relative bound, isovalues, qmax, far bound factor[, merge])
    ("normal", (19, 23, 21), 3, 8, 3e-2, 3, 32767, 0),
    ("normal", (9, 12, 17), 2, 4, 0.0, 1, 32767, 0),        # lossless: every point exact
    ("normal", (17, 9, 13), 3, 8, 2e-3, 2, 4, 0),           # most points outliers
    ("grf", (40, 40, 40), 2, 32, 1e-3, 2, 32767, 0),        # sections of 8 tiles
    ("smooth", (24, 24, 24), 4, 16, 1e-3, 2, 32767, 10),    # differentiated bounds
    ("normal", (1, 5, 70), 2, 8, 1e-2, 1, 32767, 0),        # one plane
    ("normal", (19, 23, 21), 3, 8, 3e-2, 3, 32767, 0, 2),   # merged units of up to 2 blocks per axis
    ("smooth", (40, 40, 40), 3, 8, 1e-3, 2, 32767, 0, 3),   # merged, mixed signatures
    ("grf", (40, 40, 40), 2, 8, 1e-3, 0, 32767, 0, 4),      # merged, no candidates: one signature
    ("normal", (1, 5, 70), 2, 8, 1e-2, 1, 32767, 0, 3),     # merged along x only
]


def _field(kind, shape, seed=3):
    if kind == "normal":
        return np.random.default_rng(seed).standard_normal(shape).astype(np.float32)
    if kind == "grf":
        return np.ascontiguousarray(inputs.grf(max(shape), 0.3)[: shape[0], : shape[1], : shape[2]])
    if kind == "smooth":
        return np.ascontiguousarray(inputs.gaussians(max(shape), seed=5)[: shape[0], : shape[1], : shape[2]])
    raise KeyError(kind)


def _signature(f, lo, hi, u):
    blk = f[lo[0]: hi[0] + 1, lo[1]: hi[1] + 1, lo[2]: hi[2] + 1]
    return tuple(bool(blk.min() < k <= blk.max()) for k in u)


@pytest.mark.parametrize("case", CASES,
                         ids=lambda c: f"{c[0]}-{'x'.join(map(str, c[1]))}-L{c[2]}-B{c[3]}" + (
                             f"-M{c[8]}" if len(c) > 8 else ""))
def test_independent_reader_recovers_the_oracle(case):
    kind, shape, nL, B, rel, nk, qmax, far = case[:8]
    merge = case[8] if len(case) > 8 else 0
    f = _field(kind, shape)
    e = inputs.abs_error_bound(rel, f)
    isos = list(np.quantile(f, np.linspace(0.25, 0.75, nk)).astype(np.float32))
    isos = isos + isos[:1]                        # a duplicate, dropped in the header
    r = oracle.compress(f, e, isos, levels=nL, block=B, qmax=qmax, error_bound_far=far * e, merge=merge)
    S = Stream(r["stream"])

    # header
    assert (S.magic, S.version) == (0x31524843, 1)
    assert S.dims == f.shape and (S.nL, S.B, S.qmax) == (nL, B, qmax)
    u = sorted(set(float(k) for k in isos))
    assert S.K == len(u) and S.iso[: S.K] == u and not any(S.iso[S.K:])
    assert S.e == e and S.vmin == f.min() and S.vmax == f.max()
    nb = tuple(max(1, -(-(n - 1) // B)) for n in f.shape)
    assert S.nb == nb
    assert S.merged == (merge > 1)
    if S.merged:
        # the units tile the block grid, each a rectangle of at most `merge`
        # blocks per axis whose blocks share one index signature
        owner = np.full(nb, -1)
        for b in range(S.nblocks):
            b0, b1 = S.box(b)
            assert all(0 <= b0[a] < b1[a] <= nb[a] and b1[a] - b0[a] <= S.mb[a] <= merge for a in range(3))
            assert (owner[b0[0]: b1[0], b0[1]: b1[1], b0[2]: b1[2]] == -1).all()
            owner[b0[0]: b1[0], b0[1]: b1[1], b0[2]: b1[2]] = b
            sigs = set()
            for z in range(b0[0], b1[0]):
                for y in range(b0[1], b1[1]):
                    for x in range(b0[2], b1[2]):
                        lo = [B * z, B * y, B * x]
                        hi = [min(lo[a] + B, f.shape[a] - 1) for a in range(3)]
                        sigs.add(_signature(f, lo, hi, sorted(set(float(k) for k in isos))))
            assert len(sigs) == 1, b
        assert (owner >= 0).all()
        assert S.merge == merge
        assert S.mb == tuple(max(S.box(b)[1][a] - S.box(b)[0][a] for b in range(S.nblocks)) for a in range(3))
        assert S.payload == 256 + 16 * S.nblocks * nL + 16 * S.nblocks + 32 * S.nblocks
    else:
        assert S.nblocks == nb[0] * nb[1] * nb[2]
        assert S.payload == 256 + 16 * S.nblocks * nL + 16 * S.nblocks
    assert S.flags & 1 == (e == 0)
    assert (S.flags >> 1) & 1 == (far > 0)
    if far:
        assert S.e_far == far * e
    else:
        assert S.e_far == 0 and S.far_inv == 0 and S.far_step == 0
    assert S.hdr_sum == _checksum(S.s[:252])
    assert S.tab_sum == _checksum(S.s[256: S.payload])
    assert S.nO == int((r["flags"] & 1).sum()) and S.nC == int((r["flags"] >> 1).sum())

    # every section
    q, ex, xv = S.decode()
    assert np.array_equal(q, r["q"])
    assert np.array_equal(ex, r["flags"] != 0)
    assert np.array_equal(xv[ex], f.view(np.uint32)[ex])

    # block records: min and max of the reconstruction over the closed extent
    for b in range(S.nblocks):
        lo, hi = S.extent(b)
        blk = r["xr"][lo[0]: hi[0] + 1, lo[1]: hi[1] + 1, lo[2]: hi[2] + 1]
        rec = 256 + 16 * S.nblocks * nL + 16 * b
        assert S.f32(rec) == blk.min() and S.f32(rec + 4) == blk.max()
        act = S.u32(rec + 12)
        if far:
            crosses = any(f[lo[0]: hi[0] + 1, lo[1]: hi[1] + 1, lo[2]: hi[2] + 1].min() < k
                          <= f[lo[0]: hi[0] + 1, lo[1]: hi[1] + 1, lo[2]: hi[2] + 1].max() for k in u)
            assert act == int(crosses), b
        else:
            assert act == 0


def test_reader_rejects_a_moved_section():
    """The reader is not vacuous: the same stream with two adjacent sections'
    table entries swapped fails its order check."""
    f = _field("normal", (19, 23, 21))
    r = oracle.compress(f, 0.05, [0.0], levels=3, block=8)
    s = bytearray(r["stream"])
    a, b = 256, 256 + 16
    s[a: a + 16], s[b: b + 16] = s[b: b + 16], s[a: a + 16]
    with pytest.raises(AssertionError):
        Stream(s).decode()
