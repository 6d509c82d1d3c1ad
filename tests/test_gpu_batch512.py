"""The 512-solve batch workload (seeded sweep, M = 22..1995, 32 times each)
through the serving executor in the launch configuration bench.py times
(4 slots, octave batches, grouped eigensolves), with sampled solves checked
element by element against the oracle: the smallest, the median and the two
largest problems (U(t) and the averaged probabilities within 1e-10,
quasienergies within 1e-10 normwise); every solve reports convergence and
its probability columns sum to one.
"""
import numpy as np
import pytest

import oracle
from workloads import cfg3_batch
from gpu_util import require_gpu, log

pytestmark = pytest.mark.gpu


def test_batch512_executor_against_oracle():
    torch, mmf = require_gpu()
    from paper_2005_03426_amd import serve
    items = cfg3_batch()
    reqs = [serve.Request(rid=k, arrival=0.0, problem=p, times=ts, t0=t0) for k, (p, ts, t0) in enumerate(items)]
    log("batch512 through the executor")
    ex = serve.Executor(slots=4)
    done = ex.run(reqs)
    torch.cuda.synchronize()
    assert len(done) == 512 and not ex.rejected
    assert max(ex.batches) > 1
    for r in done:
        assert int(r.result["info"].item()) == 0
        assert float((r.result["P"].sum(dim=0) - 1.0).abs().max()) < 1e-12
    by_rid = {r.rid: r for r in done}
    dims = np.array([by_rid[k].result["M"] for k in range(512)])
    order = np.argsort(dims, kind="stable")
    for k in (order[0], order[len(order) // 2], order[-2], order[-1]):
        p, ts, t0 = items[k]
        res = by_rid[int(k)].result
        log(f"oracle check of request {k} (M={dims[k]})")
        H = oracle.build_floquet(p)
        wo, Vo = oracle.eigh(H)
        assert np.abs(res["w"].cpu().numpy() - wo).max() <= 1e-10 * max(1.0, np.abs(wo).max())
        Uo = oracle.evolve(p, Vo, wo, t0, ts)
        assert np.abs(res["U"].cpu().numpy() - Uo).max() < 1e-10
        Po = oracle.avg_prob(p, Vo)
        assert np.abs(res["P"].cpu().numpy() - Po).max() < 1e-10
