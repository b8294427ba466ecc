"""The launch-shape autotuner through the C ABI."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def test_autotune_single_instance_picks_the_fastest_candidate():
    import paper_2104_03573_amd as M
    w = W.film(N=1_000_000)
    r = M.tune(w, precision=32, n_probe=1 << 17, reps=2)
    tim = r["timings_ms"]
    _say(f"[autotune film] block {r['block']} refill {r['refill']}; best {tim.min():.3f} ms, "
         f"worst {tim.max():.3f} ms")
    assert len(tim) == M.TUNE_CANDIDATES
    small = np.array([M.tune_candidate(c)[0] <= 256 for c in range(M.TUNE_CANDIDATES)])
    assert np.all(np.isfinite(tim[small])) and np.all(tim[small] > 0)
    assert np.all(np.isinf(tim[~small]))          # the film kernel takes at most 256 threads
    c = int(np.argmin(tim))
    assert (r["block"], r["refill"]) == M.tune_candidate(c)


def test_autotune_batched_sweep():
    import paper_2104_03573_amd as M
    ws = W.film_sweep(scale=0.02)
    r = M.tune(ws, precision=32, n_probe=sum(w["problem"]["N"] for w in ws) // 4, reps=1)
    tim = r["timings_ms"]
    _say(f"[autotune sweep] block {r['block']} refill {r['refill']}; best {tim.min():.3f} ms, worst {tim.max():.3f} ms")
    small = np.array([M.tune_candidate(c)[0] <= 256 for c in range(M.TUNE_CANDIDATES)])
    assert np.all(np.isfinite(tim[small]))
    assert (r["block"], r["refill"]) == M.tune_candidate(int(np.argmin(tim)))


def test_autotune_wide_transient_kernel_takes_every_block_size():
    """The transient bump's FP32 snapshot tally (100 bins x 200 times) only fits the LDS in FP32
    for a whole workgroup, which then may have up to 1024 threads."""
    import paper_2104_03573_amd as M
    w = W.transient_bump(N=400_000)
    r = M.tune(w, precision=32, n_probe=400_000, reps=1)
    tim = r["timings_ms"]
    _say(f"[autotune transient] block {r['block']} refill {r['refill']}; best {tim.min():.3f} ms, "
         f"worst {tim.max():.3f} ms")
    assert np.all(np.isfinite(tim))
    assert (r["block"], r["refill"]) == M.tune_candidate(int(np.argmin(tim)))


def test_tuned_shape_changes_no_count():
    """Any shape the tuner may pick traces the same particles into the same integer counts."""
    import paper_2104_03573_amd as M
    w = W.film(N=100_000)
    r = M.tune(w, precision=32, n_probe=1 << 15, reps=1)
    a = M.run(w, precision=32, block=r["block"], refill=r["refill"])
    b = M.run(w, precision=32, block=64, refill=1)
    assert a["counts"] == b["counts"]
    assert a["kappa"] == pytest.approx(b["kappa"], rel=1e-9)
