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
    assert np.all(np.isfinite(tim)) and np.all(tim > 0)
    c = int(np.argmin(tim))
    assert (r["block"], r["refill"]) == M.tune_candidate(c)


def test_autotune_batched_sweep():
    import paper_2104_03573_amd as M
    ws = W.film_sweep(scale=0.02)
    r = M.tune(ws, precision=32, n_probe=sum(w["problem"]["N"] for w in ws) // 4, reps=1)
    tim = r["timings_ms"]
    _say(f"[autotune sweep] block {r['block']} refill {r['refill']}; best {tim.min():.3f} ms, worst {tim.max():.3f} ms")
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
