"""Host model of the plan layout and of every event-array index the kernels
form (CPU only, no GPU, no library call).

The plan stores a batch's events in arrays of `slots` entries (dt, tau, d,
and gsd for per-pair decays); per window it keeps `begin` and `n`.  This
file restates, from the kernels' index arithmetic, every slot a kernel can
read or write for a given plan, and checks that each lies in [0, slots).
The model follows the sources line by line in what it indexes (not in what
it computes): prepare_kernel (mdhp_api.hip), team_eval and slow_decay_sums
of the lane-major kernels (mdhp_lpc.hip), eval_window and slow_decay_sums of
the lane-per-dimension kernels (mdhp_shared.hip), and eval_window_pair
(mdhp_pair.hip).

The plan of test_chunk_boundaries_wide (M = 20, first window empty) is the
case whose GPU run met an illegal address under a layout that put `dt` at
the start of one allocation: the carry pass of eval_window prefetched
slot begin + j0 + jr with jr = -1 - lane for a window without events
(guarded only by jr < len), i.e. up to one group of floats before the
window's first slot, before the array itself when the window is the plan's
first.  The model of that guard is kept below to show it reaching index -1.
"""

import numpy as np
import pytest

BLOCK = 256          # threads of the workgroup kernels
LPC_BLOCK = 256      # lane-major workgroup (4 wavefronts)
BIG_WINDOW = 1024    # default lane-major team threshold
K_AHEAD = 4          # lane-major loads in flight (for_steps)


def lanes_for(M):
    p = 4
    while p < M:
        p <<= 1
    return p


def lane_team(n, big_min):
    return LPC_BLOCK if n >= big_min else 64


def plan_layout(counts, M, beta_mode, big_min=BIG_WINDOW):
    """(begin[W], slots, lane_major) as mdhp_plan_create lays the events out."""
    counts = np.asarray(counts, np.int64)
    lane_major = beta_mode == 0 and M <= 16
    if not lane_major:
        off = np.concatenate([[0], np.cumsum(counts)])
        return off[:-1], int(off[-1]), False
    begin = np.zeros(len(counts), np.int64)
    acc = 0
    for w, n in enumerate(counts):
        L = lane_team(int(n), big_min)
        begin[w] = acc
        acc += L * ((int(n) + L - 1) // L)
    return begin, acc, True


class Touch:
    """Collects the smallest and largest index formed per array."""

    def __init__(self):
        self.lo, self.hi = {}, {}

    def add(self, name, idx):
        idx = np.asarray(idx, np.int64).ravel()
        if idx.size == 0:
            return
        self.lo[name] = min(self.lo.get(name, idx.min()), idx.min())
        self.hi[name] = max(self.hi.get(name, idx.max()), idx.max())

    def check(self, lengths):
        for name in self.lo:
            assert self.lo[name] >= 0, f"{name}: index {self.lo[name]} below 0"
            assert self.hi[name] < lengths[name], \
                f"{name}: index {self.hi[name]} past length {lengths[name]}"


def touch_prepare(tc, counts, M, beta_mode, big_min=BIG_WINDOW):
    begin, slots, lane_major = plan_layout(counts, M, beta_mode, big_min)
    off = np.concatenate([[0], np.cumsum(counts)])
    for w, n in enumerate(counts):
        n = int(n)
        if n == 0:
            continue
        k = np.arange(n)
        i = off[w] + k
        tc.add("t_in", i)
        tc.add("t_in", i[1:] - 1)
        if lane_major:
            L = lane_team(n, big_min)
            c = (n + L - 1) // L
            dst = begin[w] + L * (k % c) + k // c
        else:
            dst = i
        tc.add("slot", dst)
    tc.add("t_in", off[1:][np.asarray(counts) > 0] - 1)  # the window's last event (end gap)


def touch_lpc(tc, counts, M, big_min=BIG_WINDOW):
    """team_eval: lane t of a team of T lanes reads slots begin + t + j T for
    the steps j < c of its chunk (for_steps loads only j < c), the pending
    walk j < len, and slow_decay_sums j < c."""
    begin, slots, _ = plan_layout(counts, M, 0, big_min)
    order = np.argsort(-np.asarray(counts), kind="stable")
    n_big = int(np.sum(np.asarray(counts) >= big_min))
    for q, w in enumerate(order):
        n = int(counts[w])
        T = LPC_BLOCK if q < n_big else 64  # the kernel's team by queue position
        assert T == lane_team(n, big_min), "team and layout disagree"
        c = (n + T - 1) // T
        t = np.arange(T)
        if c == 0:
            continue
        steps = np.arange(c)
        tc.add("slot", begin[w] + t[:, None] + steps[None, :] * T)
        ln = np.clip(n - t * c, 0, c)
        for lane in range(T):
            if ln[lane] > 0:
                tc.add("slot", begin[w] + lane + np.arange(ln[lane]) * T)


def touch_shared(tc, counts, M, old_prefetch_guard=False):
    """eval_window (16 < M <= 64): group grp of P lanes owns events
    [j0, j0 + len) of the window; the carry pass prefetches backwards, the
    intensity pass forwards, slow_decay_sums forwards."""
    P = lanes_for(M)
    G = BLOCK // P
    begin, slots, _ = plan_layout(counts, M, 0)
    lane = np.arange(P)
    for w, n in enumerate(counts):
        n = int(n)
        c = (n + G - 1) // G
        for grp in range(G):
            j0 = min(grp * c, n)
            ln = min(j0 + c, n) - j0
            nsub = (c + P - 1) // P
            # Carry pass: prefetch, then the loop's prefetch of sub-batch bb - 1.
            jr = (nsub - 1) * P + (P - 1 - lane)
            ok = (jr < ln) if old_prefetch_guard else ((jr >= 0) & (jr < ln))
            tc.add("slot", begin[w] + j0 + jr[ok])
            for bb in range(nsub - 1, -1, -1):
                jr = jr - P
                if bb > 0:
                    tc.add("slot", begin[w] + j0 + jr[jr < ln])
            # Intensity pass.
            nblk = (ln + P - 1) // P
            jl = lane.copy()
            tc.add("slot", begin[w] + j0 + jl[jl < ln])
            for blk in range(nblk):
                jl = jl + P
                if blk + 1 < nblk:
                    tc.add("slot", begin[w] + j0 + jl[jl < ln])
            # Slow-decay sums.
            for sb in range(nsub):
                j = sb * P + lane
                tc.add("slot", begin[w] + j0 + j[j < ln])


def touch_pair(tc, counts, M):
    """eval_window_pair: chunk grp, batches of B events, loads jl < len."""
    P = lanes_for(M)
    G = BLOCK // P
    B = P if P < 16 else 16
    begin, slots, _ = plan_layout(counts, M, 1)
    lane = np.arange(P)
    for w, n in enumerate(counts):
        n = int(n)
        c = (n + G - 1) // G
        for grp in range(G):
            j0 = min(grp * c, n)
            ln = min(j0 + c, n) - j0
            nb = (c + B - 1) // B
            for bb in range(nb):
                jl = bb * B + (lane & (B - 1))
                tc.add("slot", begin[w] + j0 + jl[jl < ln])


WIDE_COUNTS = [0, 1, 2, 3, 7, 8, 9, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511,
               512, 513, 1023, 1024, 1025, 2047, 2049, 4100]
LANE_COUNTS = [0, 1, 2, 63, 64, 65, 127, 128, 129, 640, 641, 1023, 1024, 1025, 1279, 4095, 4096,
               4097]


def _lengths(counts, M, beta_mode, big_min=BIG_WINDOW):
    _, slots, _ = plan_layout(counts, M, beta_mode, big_min)
    return {"slot": slots, "t_in": int(np.sum(counts))}


def test_wide_plan_of_the_fault_reads_no_slot_before_its_arrays():
    counts = WIDE_COUNTS
    assert sum(counts) == 14274
    tc = Touch()
    touch_prepare(tc, counts, 20, 0)
    touch_shared(tc, counts, 20)
    tc.check(_lengths(counts, 20, 0))


def test_former_prefetch_guard_reads_before_the_first_window():
    """The guard the carry pass had: an empty first window reads slot -1 and
    below (one group of P = 32 lanes: down to -32)."""
    tc = Touch()
    touch_shared(tc, WIDE_COUNTS, 20, old_prefetch_guard=True)
    assert tc.lo["slot"] == -32
    with pytest.raises(AssertionError, match="below 0"):
        tc.check(_lengths(WIDE_COUNTS, 20, 0))


@pytest.mark.parametrize("M", [17, 20, 32, 33, 48, 64])
@pytest.mark.parametrize("first_empty", [True, False])
def test_shared_plans_in_bounds(M, first_empty):
    rng = np.random.default_rng(M)
    counts = list(rng.integers(0, 3000, 40))
    counts[0] = 0 if first_empty else counts[0]
    counts[-1] = 0
    tc = Touch()
    touch_prepare(tc, counts, M, 0)
    touch_shared(tc, counts, M)
    tc.check(_lengths(counts, M, 0))


@pytest.mark.parametrize("M", [1, 4, 5, 8, 16])
@pytest.mark.parametrize("big_min", [512, 1024, 4096, 2 ** 31 - 1])
def test_lane_major_plans_in_bounds(M, big_min):
    counts = LANE_COUNTS + [3, 0, 20000]
    tc = Touch()
    touch_prepare(tc, counts, M, 0, big_min)
    touch_lpc(tc, counts, M, big_min)
    tc.check(_lengths(counts, M, 0, big_min))


@pytest.mark.parametrize("M", [1, 3, 16, 32])
def test_pair_plans_in_bounds(M):
    counts = [0] + WIDE_COUNTS[1:] + [0]
    tc = Touch()
    touch_prepare(tc, counts, M, 1)
    touch_pair(tc, counts, M)
    tc.check(_lengths(counts, M, 1))


def test_large_window_clip_in_bounds():
    """Windows at the 50,000-event clip of the M = 64 workload."""
    counts = [50000, 0, 49999, 500, 50000]
    tc = Touch()
    touch_prepare(tc, counts, 64, 0)
    touch_shared(tc, counts, 64)
    tc.check(_lengths(counts, 64, 0))
