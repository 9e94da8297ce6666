"""Host-side model of the stream solve's slot schedule (continuous batching).

The device refill rule: after every pass, the slots that want work (idle, or
whose snapshot converged, failed or used max_iter steps) take the next
snapshots of the stream in slot order.  This model replays that rule on
random per-snapshot iteration counts and checks what the host loop of
mase_solve_stream relies on:

* every snapshot enters exactly one slot, in stream order, and leaves after
  min(its iterations, max_iter) passes;
* the number of passes never exceeds ceil(n_total * max_iter / S) + max_iter,
  the bound the host uses (plus one pass queued ahead) to detect a stream that
  does not drain.
"""
import numpy as np
import pytest


def simulate(S, need, max_iter):
    n = len(need)
    slot = [-1] * S
    done_at = [-1] * n
    left = [0] * S
    nxt = 0
    passes = 0

    def refill():
        nonlocal nxt
        for s in range(S):  # slot order, like the device's prefix count
            if slot[s] < 0 and nxt < n:
                slot[s] = nxt
                left[s] = min(need[nxt], max_iter)
                nxt += 1

    refill()
    while any(x >= 0 for x in slot):
        passes += 1
        for s in range(S):
            if slot[s] >= 0:
                left[s] -= 1
                if left[s] == 0:
                    done_at[slot[s]] = passes
                    slot[s] = -1
        refill()
    return passes, done_at, nxt


@pytest.mark.parametrize("seed", range(20))
def test_stream_schedule_bound_and_coverage(seed):
    rng = np.random.default_rng(seed)
    S = int(rng.integers(1, 17))
    n = int(rng.integers(0, 200))
    max_iter = int(rng.integers(1, 11))
    need = rng.integers(1, 15, size=n).tolist()
    passes, done_at, taken = simulate(S, need, max_iter)
    assert taken == n
    assert all(d > 0 for d in done_at)
    bound = (n * max_iter + S - 1) // S + max_iter
    assert passes <= bound, (S, n, max_iter, passes, bound)
    # every slot-pass while the stream is not exhausted does useful work
    assert passes >= -(-sum(min(x, max_iter) for x in need) // S)


def test_stream_schedule_adversarial_tail():
    # one long snapshot entering last keeps the stream alive max_iter passes
    # after the queue has emptied: the bound's second term
    S, max_iter = 4, 10
    need = [1] * 40 + [10]
    passes, _, _ = simulate(S, need, max_iter)
    assert passes == 10 + 10
    assert passes <= (len(need) * max_iter + S - 1) // S + max_iter
