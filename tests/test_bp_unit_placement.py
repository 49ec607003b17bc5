"""CPU emulation of how the eight-fold symmetric back-projector
(k_backproject_sym8) hands out its work units: the launch's grid size (the
back-projector share of the CUs), the relabelling of each block's rounds so
that the blocks of one XCD take a contiguous run of items, and the order of
a slice's units over the first-quadrant tile pairs.

The integer arithmetic is replayed as the kernel and its launcher compute
it (the back-projector relabels its units when every slice of the launch
is eight-fold symmetric; other launches take the units in slot order).  The test checks, for image sizes from one tile to 2048 pixels, batches
of several slices and every back-projector share the schedule accepts:
  * every (slice, unit) item is processed exactly once, and every block
    processes as many items as it would without the relabelling;
  * a slice's units cover every first-quadrant tile pair (a, b), a <= b,
    exactly once, each orbit's tiles in range;
  * at 512 x 512 with the default share, each XCD's 16 units form one
    4 x 4 block of tile pairs or two diagonal blocks.
"""
import pytest


def sym8_units(n):
    nq = n // 32
    return nq * (nq - 1) // 2 + (nq + 1) // 2


def sym_bp_grid(norb, pct, ncu=256):
    cap = max(1, ncu * pct // 100) if pct > 0 else (ncu // 2 if norb <= ncu else ncu)
    rounds = (norb + cap - 1) // cap
    return (norb + rounds - 1) // rounds


def xcd_item(b, r, G, N):
    x, R = b & 7, N // G
    rem = N - R * G
    off = 0
    for y in range(x):
        off += R * ((G + 7 - y) >> 3) + ((rem + 7 - y) >> 3)
    return off + r * ((G + 7 - x) >> 3) + (b >> 3)


def unit_orbits(u, nq):
    """(a, b) tile pairs of unit u: one off-diagonal pair, or one or two
    diagonal tiles (a, a)."""
    nb = (nq + 3) >> 2
    r = u
    for A in range(nb):
        ha = min(4, nq - 4 * A)
        nh = ha * (ha - 1) // 2
        if r < nh:
            a = 0
            while r >= ha - 1 - a:
                r -= ha - 1 - a
                a += 1
            return [(4 * A + a, 4 * A + a + 1 + r)]
        r -= nh
        if r < (ha + 1) // 2:
            d0 = 4 * A + 2 * r
            return [(d0, d0), (d0 + 1, d0 + 1)][:min(2, nq - d0)]
        r -= (ha + 1) // 2
    for A in range(nb):
        ha = min(4, nq - 4 * A)
        for B in range(A + 1, nb):
            hb = min(4, nq - 4 * B)
            if r < ha * hb:
                return [(4 * A + r // hb, 4 * B + r % hb)]
            r -= ha * hb
    raise AssertionError(f"unit {u} beyond the slice's units")


def blocks_items(G, N):
    """Items each block processes, in its rounds (the kernel's loop)."""
    out = []
    for b in range(G):
        items, slot, rnd = [], b, 0
        while slot < N:
            items.append(xcd_item(b, rnd, G, N))
            slot += G
            rnd += 1
        out.append(items)
    return out


@pytest.mark.parametrize("ncu", [256, 304, 80])
@pytest.mark.parametrize("npairs", [1, 2, 3, 8])
def test_every_item_once_and_the_same_work_per_block(ncu, npairs):
    for n in (32, 64, 96, 160, 256, 384, 512, 768, 1024, 2048):
        N = sym8_units(n) * npairs
        for pct in [0] + list(range(10, 401, 15)) + [400]:
            G = sym_bp_grid(N, pct, ncu)
            per_block = blocks_items(G, N)
            seen = sorted(i for items in per_block for i in items)
            assert seen == list(range(N)), (n, npairs, pct, G)
            for b, items in enumerate(per_block):
                assert len(items) == len(range(b, N, G)), (n, npairs, pct, b)


@pytest.mark.parametrize("n", [32, 64, 96, 128, 160, 224, 256, 384, 512, 768, 1024, 2048])
def test_units_cover_every_tile_pair_once(n):
    nq = n // 32
    got = []
    for u in range(sym8_units(n)):
        orbits = unit_orbits(u, nq)
        assert 1 <= len(orbits) <= 2
        if len(orbits) == 2:
            assert all(a == b for a, b in orbits)
        for a, b in orbits:
            assert 0 <= a <= b < nq
            got.append((a, b))
    assert sorted(got) == [(a, b) for a in range(nq) for b in range(a, nq)]


def test_512_units_of_an_xcd_are_one_block_of_tiles():
    n = 512
    nq, N = n // 32, sym8_units(n)
    G = sym_bp_grid(N, 0)
    assert G == N == 128
    per_xcd = {}
    for b, items in enumerate(blocks_items(G, N)):
        for i in items:
            per_xcd.setdefault(b & 7, []).extend(unit_orbits(i, nq))
    for x, tiles in per_xcd.items():
        blocks = {(a // 4, b // 4) for a, b in tiles}
        diag = all(A == B for A, B in blocks)
        assert (len(blocks) == 1 and not diag) or (diag and len(blocks) == 2), (x, blocks)
