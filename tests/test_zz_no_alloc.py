"""The allocation-free batched trace (mcbte_trace_batch_static, for callers that cannot allocate):
its work queue is the library's static device array, filled by a setup kernel on the stream.  It
must give what mcbte_trace_batch gives with a caller-owned queue: every integer counter equal,
the FP64 sums to the rounding of the atomics' order, on two calls in a row (the second with fewer
instances and particles, so the shared array holds a smaller table over the larger one's
leftovers), and refuse more instances than the array holds."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _films(n_inst, scale, seed):
    out = []
    for i in range(n_inst):
        d = 10.0 ** (-8.0 + 2.5 * i / max(1, n_inst - 1))
        w = W.film(N=int(scale * (2000 + 1500 * i)), d=d, T=(100.0, 300.0, 200.0)[i % 3], seed=seed)
        w["instance"] = 5 + 3 * i
        out.append(w)
    return out


@pytest.mark.parametrize("precision", [64, 32])
def test_static_batched_trace_equals_the_queued_one(precision):
    import torch
    import paper_2104_03573_amd as M
    for ws in (_films(7, 1.0, W.SEED_BASE + 41), _films(3, 0.5, W.SEED_BASE + 42)):
        print(f"[no-alloc] precision {precision}, {len(ws)} instances, N {[w['problem']['N'] for w in ws]}",
              flush=True)
        tabs = [M.Tables(w) for w in ws]
        ns = [w["problem"]["N"] for w in ws]
        ids = [w["instance"] for w in ws]
        run = M.make_run(int(ws[0]["seed"]), precision)
        t_q = [t.new_tally() for t in tabs]
        queue = torch.zeros(M.batch_queue_bytes(len(ws)), dtype=torch.uint8, device="cuda")
        M.trace_batch(tabs, ns, ids, t_q, run, queue)
        t_s = [t.new_tally() for t in tabs]
        M.trace_batch_static(tabs, ns, ids, t_s, run)
        for t, a, b, n in zip(tabs, t_q, t_s, ns):
            ra, rb = M.tally(t, a), M.tally(t, b)
            assert ra["counts"]["particles"] == n
            assert np.array_equal(ra["counts_raw"], rb["counts_raw"])
            xa, xb = t.raw(a), t.raw(b)
            assert np.abs(xa - xb).max() <= 1e-12 * np.abs(xa).max()
            assert np.allclose(ra["moments"], rb["moments"], rtol=1e-12, atol=1e-12 * np.abs(ra["moments"]).max())


def test_static_batched_trace_refuses_more_instances_than_it_holds():
    import paper_2104_03573_amd as M
    w = W.film(N=10)
    t = M.Tables(w)
    n = M.mcbte.STATIC_MAX_INSTANCES + 1
    tallies = [t.new_tally() for _ in range(n)]
    with pytest.raises(M.MCBTEError) as e:
        M.trace_batch_static([t] * n, [10] * n, list(range(n)), tallies, M.make_run(1, 64))
    assert e.value.status == M.mcbte.ELIMIT
