"""GPU tests of the serving loop: results are the same alone and in the mix,
and served ridge solves reach the closed-form optimum's objective to 1e-4."""

import numpy as np
import pytest

import workloads as wl
from oracle import bsadmm_oracle as o

pytestmark = pytest.mark.gpu


def _jobs():
    from paper_1409_0940_amd.serving import Job
    reqs = [r for r in wl.serving_stream(256) if r.n <= 12000 and r.s <= 2048][:6]
    jobs = []
    for r in reqs:
        inp = wl.make_inputs(wl.request_workload(r))
        jobs.append(Job(r.rid, 0.0, r, inp))
    return jobs


def test_same_result_alone_and_in_the_mix():
    from paper_1409_0940_amd.serving import GpuExecutor, Scheduler
    jobs = _jobs()
    assert len({(j.spec.d, j.spec.loss) for j in jobs}) >= 3
    ex = GpuExecutor("bf16x3", max_streams=4)
    mix = Scheduler(ex, 64 << 30, max_active=4, max_iters=300).run(jobs, time_scale=0.0)
    assert max(len([1 for r in mix.values()]), 0) == len(jobs)
    for j in jobs:
        ex1 = GpuExecutor("bf16x3", max_streams=1)
        alone = Scheduler(ex1, 64 << 30, max_active=1, max_iters=300).run([j], time_scale=0.0)
        a, m = alone[j.rid], mix[j.rid]
        assert a.status == m.status == "ok"
        assert a.iters == m.iters, j.rid
        assert np.array_equal(a.coef, m.coef), j.rid


@pytest.mark.parametrize("rho_adapt", [None, (10, 5.0, 2.0)], ids=["fixed_rho", "adaptive_rho"])
def test_served_ridge_solves_reach_the_optimum(rho_adapt):
    from paper_1409_0940_amd.serving import GpuExecutor, Scheduler
    jobs = [j for j in _jobs() if j.spec.loss == "squared"]
    assert jobs
    res = Scheduler(GpuExecutor("bf16x3", 4, rho_adapt=rho_adapt), 64 << 30, max_active=4,
                    max_iters=300).run(jobs, time_scale=0.0)
    for j in jobs:
        X, Y, W, b = j.inputs
        Z = o.rff(X, W, b)
        fstar = o.objective("squared", Z, Y, o.ridge_closed_form(Z, Y, j.spec.lam), j.spec.lam)
        f = o.objective("squared", Z, Y, res[j.rid].coef, j.spec.lam)
        assert (f - fstar) / fstar <= 1e-4, (j.rid, f, fstar)
