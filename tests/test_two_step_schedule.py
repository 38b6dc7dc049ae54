"""CPU check of the narrow two-step sweep's schedule (sweep_narrow2_kernel):
stage A (step t) writes row groups of 64 / nx rows into a ring of eight
groups in LDS, one group per iteration; stage B (step t + 1) starts at
iteration min(L - 1, nA) and runs its group b at
jB(b) = max(min(b + L, nA), jB(0) + b), reading rows of stage A's groups up
to two rows past its next group. With one barrier per iteration, every ring
read must find the group it wants written in an earlier iteration and not
yet overwritten (the slot stage A writes in the same iteration must hold no
group stage B still reads), and every row stage B stores must depend only on
rows stage A computed exactly (y - 2 .. y + 2 inside the channel). The same
index arithmetic as the kernel: row groups counted from
yA0 = max(y0 - 2, 0), rows clamped to [yA0, yA1 - 1] before the ring
lookup, L = 3 + 2 // (64 // nx)."""
import pytest

RING = 8


def check_strip(ny, nx, y0, y1, lag=None):
    tyw = 64 // nx
    lag = 3 + 2 // tyw if lag is None else lag
    assert lag <= RING
    ya0, ya1 = max(y0 - 2, 0), min(y1 + 2, ny)
    na = (ya1 - ya0 + tyw - 1) // tyw
    nb = (y1 - y0 + tyw - 1) // tyw
    slot = {}  # ring slot -> (group, iteration written)

    def pulled_rows(y):
        yc = min(max(y, 0), ny - 1)
        return [min(max(r, ya0), ya1 - 1) for r in (yc - 1, yc, yc + 1)]

    def reads(rows, j):
        for y in rows:
            for r in pulled_rows(y):
                g = (r - ya0) // tyw
                held = slot.get(g % RING)
                assert held is not None and held[0] == g and held[1] < j, (ny, nx, y0, y1, j, y, r, g, held)
                # stage A's write of this iteration goes to slot j % RING
                assert j >= na or g % RING != j % RING, (ny, nx, y0, y1, j, g)

    js = min(lag - 1, na)
    jb0 = min(lag, na)

    def jb(b):
        return max(min(b + lag, na), jb0 + b)

    bnext = 0
    for j in range(max(na, jb(nb - 1) + 1)):
        if j == js:  # stage B starts: the group below its first, and its first
            reads([y0 - tyw + ly for ly in range(tyw)] + [y0 + ly for ly in range(tyw)], j)
        if bnext < nb and j == jb(bnext):  # stage B's group b assembles group b + 1
            reads([y0 + (bnext + 1) * tyw + ly for ly in range(tyw)], j)
            bnext += 1
        if j < na:
            slot[j % RING] = (j, j)
    assert bnext == nb
    for y in range(y0, y1):
        for r in range(y - 2, y + 3):
            if 0 <= r < ny:
                assert ya0 <= r < ya1


@pytest.mark.parametrize("nx", [1, 2, 4, 8, 16, 32, 64])
def test_narrow_two_step_schedule(nx):
    tyw = 64 // nx
    for ny in list(range(1, 40)) + [64, 130, 200, 511]:
        for h in sorted({tyw * k for k in range(1, 9)} | {max(tyw, 64), 16 * tyw}):
            for y0 in range(0, ny, h):
                check_strip(ny, nx, y0, min(y0 + h, ny))


def test_schedule_check_catches_a_short_lag():
    """The check itself: with stage B one iteration earlier than the
    kernel's lag, a strip of four 8-row groups reads a group stage A has
    not yet written."""
    with pytest.raises(AssertionError):
        check_strip(100, 8, 16, 48, lag=2)
