"""CPU emulation of the staging rounds of the eight-fold symmetric
back-projector (k_backproject_sym8): the index arithmetic that picks, per
wavefront and pair of views, which detector bins each of the 64 lanes stages
into LDS and which staged slots each lane's chord loop then reads.

The arithmetic is replayed in 32-bit two's-complement integers, as the
kernel computes it.  For the kernel's form the test checks, over random
per-lane bin windows (empty, partly off the detector, long enough for
several rounds):
  * every staged bin is in [0, n_det) and every slot in [0, 64);
  * each bin of each view's wavefront window is staged exactly once;
  * each lane's chord loop reads only slots staged in the same round for
    the same view, and visits each bin of its own window exactly once.
The form before the fix (an empty view's staging base taken from its
window minimum, INT_MAX, and no lower bound on the staged bin) is replayed
too: there `INT_MAX + lane` wraps to a negative bin that passes the upper
bound test, which is the out-of-range read the fix removed.
"""
import numpy as np
import pytest

INT_MAX = 2 ** 31 - 1
INT_MIN = -2 ** 31


def w32(x):
    """int32 wraparound of a Python integer."""
    return ((x + 2 ** 31) % 2 ** 32) - 2 ** 31


def rounds(jlA, jhA, jlB, jhB, two, nd, fixed=True):
    """Replay one pair of views.  jl*/jh*: per-lane windows (64 each; empty
    lane = (INT_MAX, INT_MIN)).  Returns (staged, reads): staged[(view, bin)]
    = times staged; reads[(lane, view, bin)] = times read, with the checks of
    the kernel's own conditions asserted on the way."""
    JloA = max(min(jlA), 0)
    JhiA = min(max(jhA), nd - 1)
    JloB = max(min(jlB), 0) if two else INT_MAX
    JhiB = min(max(jhB), nd - 1) if two else INT_MIN
    emA, emB = JloA > JhiA, JloB > JhiB
    packed = (emA or JhiA - JloA < 32) and (emB or JhiB - JloB < 32)
    nA = 0 if emA else (JhiA - JloA) // 64 + 1
    nB = 0 if emB else (JhiB - JloB) // 64 + 1
    nround = 1 if packed else nA + nB
    staged, reads, bad = {}, {}, []
    for rd in range(nround):
        baseA, hiA, baseB, hiB, sB = 0, INT_MIN, 0, INT_MIN, 64
        if packed:
            if fixed:
                baseA = 0 if emA else JloA
                baseB = 0 if emB else JloB
            else:
                baseA, baseB = JloA, JloB
            hiA = INT_MIN if emA else JhiA
            hiB = INT_MIN if emB else JhiB
            sB = 32
        elif rd < nA:
            baseA = JloA + 64 * rd
            hiA = min(JhiA, baseA + 63)
        else:
            baseB = JloB + 64 * (rd - nA)
            hiB = min(JhiB, baseB + 63)
            sB = 0
        slot_of = {}
        for lane in range(64):
            hb = lane >= sB
            jj = w32(baseB + (lane - sB)) if hb else w32(baseA + lane)
            ok = (jj >= 0 if fixed else True) and jj <= (hiB if hb else hiA)
            if ok:
                view = "B" if hb else "A"
                if not (0 <= jj < nd):
                    bad.append((view, jj, lane))
                    continue
                staged[(view, jj)] = staged.get((view, jj), 0) + 1
                slot_of[(view, jj)] = lane
        for lane in range(64):
            for h, view in ((0, "A"), (1, "B")):
                jl = jlB[lane] if h else jlA[lane]
                jh = jhB[lane] if h else jhA[lane]
                base = baseB if h else baseA
                hi = hiB if h else hiA
                s0 = sB if h else 0
                lo_j, hi_j = max(jl, base), min(jh, hi)
                for j in range(lo_j, hi_j + 1):
                    slot = j - base + s0
                    assert 0 <= slot < 64, (lane, view, j, slot)
                    assert slot_of.get((view, j)) == slot, (lane, view, j)
                    reads[(lane, view, j)] = reads.get((lane, view, j), 0) + 1
    return staged, reads, bad


def random_windows(rng, nd, long=False, empty_frac=0.2):
    jl = np.empty(64, dtype=np.int64)
    jh = np.empty(64, dtype=np.int64)
    start = int(rng.integers(-30, nd + 10))
    span = 200 if long else 24
    for lane in range(64):
        if rng.random() < empty_frac:
            jl[lane], jh[lane] = INT_MAX, INT_MIN
        else:
            a = start + int(rng.integers(-8, 9))
            jl[lane], jh[lane] = a, a + int(rng.integers(0, span))
    return [int(x) for x in jl], [int(x) for x in jh]


def empty_windows():
    return [INT_MAX] * 64, [INT_MIN] * 64


def expected(jl, jh, nd):
    out = set()
    for a, b in zip(jl, jh):
        for j in range(max(a, 0), min(b, nd - 1) + 1):
            out.add(j)
    return out


def check_pair(jlA, jhA, jlB, jhB, two, nd):
    staged, reads, bad = rounds(jlA, jhA, jlB, jhB, two, nd)
    assert not bad
    for view, (jl, jh) in (("A", (jlA, jhA)), ("B", (jlB, jhB))):
        if view == "B" and not two:
            assert not any(k[0] == "B" for k in staged)
            continue
        want = expected(jl, jh, nd)
        got = {j for (v, j) in staged if v == view}
        assert want <= got, view
        assert all(staged[(view, j)] == 1 for j in got)
        for lane in range(64):
            lane_want = set(range(max(jl[lane], 0), min(jh[lane], nd - 1) + 1))
            lane_got = {j for (l, v, j), c in reads.items() if l == lane and v == view}
            assert lane_got == lane_want, (view, lane)
            assert all(c == 1 for (l, v, j), c in reads.items() if l == lane and v == view)


@pytest.mark.parametrize("nd", [64, 300, 736, 888])
def test_staging_rounds_stay_in_bounds_and_cover_each_bin_once(nd):
    rng = np.random.default_rng(nd)
    for case in range(240):
        longA, longB = rng.random() < 0.3, rng.random() < 0.3
        jlA, jhA = random_windows(rng, nd, longA)
        jlB, jhB = random_windows(rng, nd, longB)
        two = rng.random() < 0.8
        kind = case % 6
        if kind == 1:
            jlA, jhA = empty_windows()
        elif kind == 2:
            jlB, jhB = empty_windows()
        elif kind == 3:
            jlA, jhA = empty_windows()
            jlB, jhB = empty_windows()
        if not two:
            jlB, jhB = [INT_MAX] * 64, [INT_MIN] * 64
        check_pair(jlA, jhA, jlB, jhB, two, nd)


def test_windows_entirely_off_the_detector_are_empty():
    nd = 128
    jl = [nd + 5] * 64
    jh = [nd + 20] * 64
    staged, reads, bad = rounds(jl, jh, [-40] * 64, [-2] * 64, True, nd)
    assert not staged and not reads and not bad


def test_pre_fix_form_reads_out_of_range_on_an_empty_view():
    """The form before the fix stages a wrapped, negative bin when a packed
    round holds an empty view: the emulation sees the read the fix removed."""
    nd = 300
    jlA, jhA = [100 + (lane % 5) for lane in range(64)], [110 + (lane % 7) for lane in range(64)]
    jlB, jhB = empty_windows()
    _, _, bad = rounds(jlA, jhA, jlB, jhB, True, nd, fixed=False)
    assert bad and all(j < 0 for _, j, _ in bad)
    _, _, bad = rounds(jlA, jhA, jlB, jhB, True, nd, fixed=True)
    assert not bad
