"""CPU replay of how the fused step's waves walk the work items of one XCD's
range (the loop at the top of k_ifcm_gather): every item of the range is
processed exactly once, by index alone (no hand-out, or a stop rule) and
with the last tenth handed out by counter in any order the waves happen to
draw their tickets.  The replay follows the kernel's arithmetic: W waves,
wave w takes items beg + w + k W for k < spw, then (with hand-out) item
beg + spw W + ticket until that passes the end of the range."""
import random

import pytest


def walk(n_it, W, handout_flag, rng, one_item_without_handout=False):
    handout = handout_flag and n_it > W
    spw = max(1, n_it * 9 // 10 // W) if handout else (n_it + W - 1) // W
    if one_item_without_handout and not handout:
        spw = 1  # a planted mistake: without hand-out each wave stops after one item
    it_dyn = spw * W
    counter = 0
    seen = []
    # each wave: a generator of the items it processes
    def wave(w):
        nonlocal counter
        k = 0
        it = w
        ticket = 0
        while it < n_it:
            if handout and k + 1 >= spw:
                ticket = counter  # the atomic add's old value
                counter += 1
            yield it
            k += 1
            if k < spw:
                it = w + k * W
            else:
                it = it_dyn + ticket if handout else n_it
    gens = [wave(w) for w in range(W)]
    live = list(range(W))
    # interleave the waves at random: a wave's next item (and its ticket) is
    # taken whenever the scheduler picks it
    while live:
        w = rng.choice(live)
        try:
            seen.append(next(gens[w]))
        except StopIteration:
            live.remove(w)
    return seen, counter


@pytest.mark.parametrize("handout", [False, True])
def test_every_item_once(handout):
    rng = random.Random(7)
    for W in (1, 2, 3, 8, 64, 256):
        for n_it in list(range(0, 3 * W + 3)) + [W * 9 + 1, W * 10, W * 37 + 5, 5000]:
            for _ in range(3):
                seen, _ = walk(n_it, W, handout, rng)
                assert sorted(seen) == list(range(n_it)), (n_it, W, handout)


def test_counter_draws_bounded():
    """The counter is drawn at most once per handed-out item plus once per
    wave (each wave's last draw finds the range empty)."""
    rng = random.Random(8)
    for W in (4, 64, 256):
        for n_it in (W + 1, 2 * W, 10 * W + 3, 50 * W):
            _, draws = walk(n_it, W, True, rng)
            spw = max(1, n_it * 9 // 10 // W)
            assert draws <= (n_it - spw * W) + W


def test_walk_without_handout_beyond_one_item_per_wave_is_caught():
    """With the mistake of a wave taking one item by index and no hand-out
    to take the rest planted in the replay, a range with more items than
    waves loses items and the check above fails."""
    rng = random.Random(9)
    seen, _ = walk(3 * 8 + 1, 8, False, rng, one_item_without_handout=True)
    assert sorted(seen) != list(range(3 * 8 + 1))
    seen, _ = walk(5, 8, False, rng, one_item_without_handout=True)
    assert sorted(seen) == list(range(5))  # fewer items than waves: no loss
