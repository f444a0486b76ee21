"""The pair schedule of the one-sided Jacobi SVT, stated on the host and
checked exhaustively over the shapes the planner can produce.

The kernels (tilt_kernels.hip: CirclePairs, InnerPairs, CrossPairs,
superblock_pair, and the rounds of jacobi_rows / jacobi_pair_rows) examine
row pairs in rounds.  Two properties carry the correctness of the SVT and
of the helpers that run the pairs of a round on several workgroups:

* every pair of rows is examined exactly once per sweep (a sweep without
  rotations then means every pair is orthogonal to the tolerance);
* the rows of one round are disjoint (so its pairs commute, and may run in
  any order, on any workgroup, with the same result).

This is the schedule written out again from those structures, not a call
into the kernels; the GPU tests cover the kernels' results.  It also checks
the pair count the kernels add to their work counters per sweep, which
the bench's work model and the sweep statistics rely on."""

import itertools

import pytest

SVT_MAX_ROWS = 256          # rows held in LDS at once (two staged super-blocks)
SVT_MAX_TILED_ROWS = 1024   # rows of a tiled working plane


def circle(r, nb_minus_1, k):
    """Pair k of round r of the circle (round-robin) ordering over
    nb_minus_1 + 1 blocks: block nb_minus_1 stays, the others turn."""
    if k == 0:
        return nb_minus_1, r
    return (r + k) % nb_minus_1, (r - k) % nb_minus_1


def block_rows(b, bs, base=0):
    return [base + b * bs + t for t in range(bs)]


def examine(rounds, bs, first_round_inside):
    """Pairs examined by a list of rounds of block pairs; asserts the rows
    of every round are disjoint.  In the first round, two-row blocks also
    examine the pair inside each block."""
    seen = []
    for i, rnd in enumerate(rounds):
        touched = set()
        for ra, rb in rnd:
            for x in ra + rb:
                assert x not in touched, ("rows of a round overlap", i, x)
                touched.add(x)
            seen += [(a, b) for a in ra for b in rb]
            if i == 0 and first_round_inside and bs == 2:
                seen += [(ra[0], ra[1]), (rb[0], rb[1])]
    return seen


def in_lds_sweep(nc, bs):
    """jacobi_rows: nc rounded up to 4 rows, nb = nc4 / bs blocks, nb - 1
    circle rounds of nb / 2 block pairs."""
    nc4 = (nc + 3) & ~3
    nb = nc4 // bs
    rounds = [[(block_rows(I, bs), block_rows(J, bs)) for I, J in (circle(r, nb - 1, k) for k in range(nb // 2))]
              for r in range(nb - 1)]
    return nc4, examine(rounds, bs, True)


def staged_pair(sb, bs, inner, base_i, base_j):
    """jacobi_pair_rows on super-blocks at rows base_i and base_j: with
    `inner`, h - 1 circle rounds run in both super-blocks at once (h block
    pairs per round), then h cross rounds, round s joining block a of the
    first with block (a + s) mod h of the second."""
    h = sb // bs
    seen = []
    if inner:
        rounds = []
        for r in range(h - 1):
            rnd = []
            for k in range(h):
                half = 1 if k >= h // 2 else 0
                I, J = circle(r, h - 1, k - half * (h // 2))
                base = base_j if half else base_i
                rnd.append((block_rows(I, bs, base), block_rows(J, bs, base)))
            rounds.append(rnd)
        seen += examine(rounds, bs, True)
    cross = [[(block_rows(a, bs, base_i), block_rows((a + s) % h, bs, base_j)) for a in range(h)] for s in range(h)]
    seen += examine(cross, bs, False)
    return seen


def tiled_sweep(nsb, sb, bs):
    """One sweep of the tiled Jacobi: nsb - 1 circle rounds over the
    super-blocks, nsb / 2 super-block pairs each (the pairs of a round touch
    disjoint super-blocks); the pairs inside the super-blocks are examined
    in round 0, where every super-block appears once.  Returns the pairs
    and the count the kernel adds to its counter per staged pair."""
    seen, counted = [], 0
    for r in range(nsb - 1):
        used = set()
        for k in range(nsb // 2):
            I, J = circle(r, nsb - 1, k)
            assert I not in used and J not in used, "super-blocks of a round overlap"
            used |= {I, J}
            seen += staged_pair(sb, bs, r == 0, I * sb, J * sb)
            counted += sb * sb + (sb * (sb - 1) if r == 0 else 0)
    return seen, counted


def assert_each_pair_once(seen, rows):
    keys = sorted((min(a, b), max(a, b)) for a, b in seen)
    assert all(a != b for a, b in keys), "a row paired with itself"
    assert len(keys) == rows * (rows - 1) // 2, (len(keys), rows)
    assert len(set(keys)) == len(keys), "a pair examined twice in a sweep"


@pytest.mark.parametrize("bs", [1, 2])
def test_in_lds_sweep_examines_each_pair_once(bs):
    for nc in list(range(1, 41)) + [97, 100, 128, 170, 255, 256]:
        nc4, seen = in_lds_sweep(nc, bs)
        assert_each_pair_once(seen, nc4)


def planner_tilings():
    """Every (super-blocks, rows per super-block) the planner's search can
    return: an even number of super-blocks, super-blocks of a multiple of 4
    rows, two of them within the LDS row limit, the plane within its limit."""
    for nsb in range(2, SVT_MAX_TILED_ROWS // 4 + 1, 2):
        for sb in range(4, SVT_MAX_ROWS // 2 + 1, 4):
            if nsb * sb <= SVT_MAX_TILED_ROWS:
                yield nsb, sb


@pytest.mark.parametrize("bs", [1, 2])
def test_tiled_sweep_examines_each_pair_once(bs):
    tilings = list(planner_tilings())
    small = [t for t in tilings if t[0] * t[1] <= 160]
    large = [(2, 128), (4, 128), (8, 128), (4, 64), (16, 64), (8, 32), (32, 32), (64, 16), (128, 8), (256, 4)]
    assert all(t in tilings for t in large)
    for nsb, sb in itertools.chain(small, large):
        seen, counted = tiled_sweep(nsb, sb, bs)
        ncp = nsb * sb
        assert_each_pair_once(seen, ncp)
        assert counted == ncp * (ncp - 1) // 2


def test_a_planted_schedule_error_is_caught():
    """The checks fail on the kinds of mistake they are there for."""
    nsb, sb, bs = 4, 8, 2
    seen, _ = tiled_sweep(nsb, sb, bs)
    with pytest.raises(AssertionError):          # one pair dropped
        assert_each_pair_once(seen[1:], nsb * sb)
    with pytest.raises(AssertionError):          # one pair twice
        assert_each_pair_once(seen + seen[:1], nsb * sb)
    with pytest.raises(AssertionError):          # a round that reuses a row
        examine([[([0, 1], [2, 3]), ([2, 3], [4, 5])]], 2, False)
