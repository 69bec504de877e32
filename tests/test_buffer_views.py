"""Host-side replica of the pair pass's buffer-view addressing.

The pass (`pair_pass_item` in cr_kernels.hip) reads theta, the packed X
operands and y through per-workgroup raw buffer views: each lane keeps a fixed
32-bit byte offset, tile m of a wave adds m times a per-view step as the scalar
offset, and a load whose offset lies at or past the view's size returns zeros
(so the prefetch of the NSET tiles past a wave's last tile needs no clamp).
This file recomputes, on the CPU and for every launch layout the library picks
(the real chunk heights, from cr_pass_layout), each lane's offsets for every
tile and prefetch and checks that

  * the view sizes and every voffset + soffset fit 32 bits (no wrap-around
    into the view),
  * every access of a tile the wave processes lies inside its view and inside
    the array the view is cut from,
  * every prefetch past the wave's last tile starts at or past the view's end.

The offset formulas restate the kernel's (lane l = 16 g + c, wave w, row map
orow = 4 g + v for FP32 and mixed, g + 4 v for FP64)."""
import math

import numpy as np
import pytest

WAVES = 4
U32 = 2 ** 32


def _cr():
    import paper_1407_7220_amd as cr
    return cr


def _ops(prec, n):
    """(element size, TW, NSET, bytes of one packed-X entry, row-map kind, theta elements per lane-row)."""
    if prec == 2:
        kb = (3 * n + 31) // 32
        nkb = (n + 1 + 15) // 16
        return 4, 4, (3 if kb + nkb <= 2 else 2), (kb + nkb) * 16, "rm4"
    esz = 8 if prec == 0 else 4
    ks = (n + 1 + 3) // 4
    nkb = 1 if ks <= 4 else 2
    q = ks + 4 * nkb
    qp = ((q * esz + 15) // 16) * 16 // esz
    return esz, (2 if prec == 0 else 4), 2, qp * esz, ("g4v" if prec == 0 else "rm4")


def _lane_rows(kind):
    g = np.arange(64)[:, None] // 16
    v = np.arange(4)[None, :]
    return 4 * g + v if kind == "rm4" else g + 4 * v          # (64 lanes, 4 values)


def _check_layout(N, n, prec, tile_rows):
    cr = _cr()
    L = cr.pass_layout(N, n, cr.Params(precision=prec, tile_rows=tile_rows))
    esz, TW, NSET, XPB, kind = _ops(prec, n)
    Nrow, ld, rpc, chunks, strips = L["Nrow"], L["ld"], L["rows_per_chunk"], L["chunks"], L["strips"]
    assert strips * 16 * TW == ld and rpc % 64 == 0 and chunks == math.ceil(Nrow / rpc)
    row_bytes = ld * esz
    theta_bytes = Nrow * ld * esz
    xp_bytes = (Nrow // 16) * 64 * XPB
    lrow = _lane_rows(kind)                                   # row of (lane, v) within a 16-row tile
    cidx = np.arange(64)[:, None] % 16
    for h in sorted({0, chunks - 1}):
        I0 = h * rpc
        I1 = min(I0 + rpc, Nrow)
        rows = I1 - I0
        assert rows >= 64 and rows % 64 == 0
        th_view, xp_view, y_view = rows * row_bytes, (rows // 16) * 64 * XPB, rows * esz
        assert th_view < U32 and xp_view < U32 and y_view < U32
        for w in range(WAVES):
            ntile = -(-(I1 - (I0 + 16 * w)) // 64)
            assert ntile >= 1
            m = np.arange(ntile + NSET)[:, None, None]
            valid = m < ntile
            # theta: one 16-byte load per (lane, v), tile step 64 rows
            th_off = (16 * w + lrow)[None] * row_bytes + (TW * cidx * esz)[None] + m * (16 * WAVES * row_bytes)
            assert (th_off + 16 < U32).all()
            assert (th_off[valid[:, 0, 0]] + 16 <= th_view).all()
            assert (th_off[~valid[:, 0, 0]] >= th_view).all()
            for J0 in sorted({0, (strips - 1) * 16 * TW}):
                assert ((I0 * ld + J0) * esz + th_off[valid[:, 0, 0]] + 16 <= theta_bytes).all()
            # packed X: XPB bytes per (tile, lane), tile step 4 tiles
            xp_off = (w * 64 + np.arange(64))[None, :] * XPB + np.arange(ntile + NSET)[:, None] * (WAVES * 64 * XPB)
            vm = np.arange(ntile + NSET) < ntile
            assert (xp_off + XPB < U32).all()
            assert (xp_off[vm] + XPB <= xp_view).all() and (xp_off[~vm] >= xp_view).all()
            assert ((I0 >> 4) * 64 * XPB + xp_off[vm] + XPB <= xp_bytes).all()
            # y (non-lazy passes): 16 bytes per lane (rows 4g..4g+3) in FP32, 8 per (lane, v) in FP64
            if esz == 4:
                y_off = (16 * w + 4 * (np.arange(64) // 16))[None, :] * 4 + np.arange(ntile + NSET)[:, None] * (64 * 4)
                ext = 16
            else:
                y_off = ((16 * w + lrow)[None] * 8 + m * (64 * 8)).reshape(ntile + NSET, -1)
                ext = 8
            assert (y_off[vm] + ext <= y_view).all() and (y_off[~vm] >= y_view).all()


def _check_reduce_views(N, n, prec, tile_rows):
    """The reduce kernel's views of the row partials (strip-major, strips x Nrow)
    and column partials (chunks x ld x (n + 1)): batches of 12 strips x G and
    16 chunks, based at the wave's first point; every offset of a batch fits 32
    bits and entries of existing strips (chunks) lie inside the view."""
    cr = _cr()
    L = cr.pass_layout(N, n, cr.Params(precision=prec, tile_rows=tile_rows))
    esz = 8 if prec == 0 else 4
    G = 16 if n + 1 <= 16 else 32
    URS, UCK = 12, 16
    Nrow, ld, strips, chunks, nc = L["Nrow"], L["ld"], L["strips"], L["chunks"], n + 1
    k = np.arange(G)
    for p in (0, 64 // G - 1):
        rvo = (k * Nrow + p) * esz
        rso = G * Nrow * esz
        cvo = (p * nc + k) * esz
        cso = ld * nc * esz
        e_r = np.arange(URS)[:, None]
        e_c = np.arange(UCK)[:, None]
        assert (rvo[None, :] + e_r * rso + esz < U32).all()
        assert (cvo[None, :] + e_c * cso + esz < U32).all()
        for s0 in range(0, strips, G * URS):
            view = min((strips - s0) * Nrow * esz, U32 - 1)
            strip = s0 + k[None, :] + G * e_r
            off = rvo[None, :] + e_r * rso
            assert (off[strip < strips] + esz <= view).all()
        for h0 in range(0, chunks, UCK):
            view = min((chunks - h0) * ld * nc * esz, U32 - 1)
            chunk = h0 + e_c + 0 * k[None, :]
            off = cvo[None, :] + e_c * cso
            assert (off[(chunk < chunks) & (k[None, :] < nc)] + esz <= view).all()


def test_reduce_views():
    for prec in (0, 1):
        for n in (1, 10, 20, 31):
            for N in (37, 5000, 20000, 65536, 1 << 20):
                for tr in (0, 64, 4096):
                    _check_reduce_views(N, n, prec, tr)


CASES = [(N, n, prec, tr)
         for prec in (0, 1, 2)
         for n in (1, 3, 10, 20, 31)
         for N in (2, 37, 64, 1000, 1700, 5000, 20000)
         for tr in (0, 64, 128, 768, 3072, 4096)
         if not (prec == 2 and n > 31)]


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "mixed"])
def test_pass_views_every_layout(prec):
    for (N, n, p, tr) in CASES:
        if p == prec:
            _check_layout(N, n, p, tr)


@pytest.mark.parametrize("N,prec", [(131072, 1), (65536, 0), (1 << 20, 1), (1 << 20, 0), (1 << 20, 2)],
                         ids=["f32-131072", "f64-65536", "f32-2^20", "f64-2^20", "mixed-2^20"])
def test_pass_views_at_the_largest_sizes(N, prec):
    """The 32-bit limits: the chunk-height cap keeps the views and every prefetch
    offset below 2^32 up to the largest supported N."""
    for n in (3, 20):
        for tr in (0, 4096):
            _check_layout(N, n, prec, tr)
