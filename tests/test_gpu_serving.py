"""Continuous batching: each result is the same alone and in the mix."""

import copy

import pytest
import torch

pytestmark = pytest.mark.gpu


def test_batched_results_equal_serial_results():
    import sys, os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from bench import make_requests
    from paper_2410_02395_amd.serve import Server, run_serial, summarize
    from paper_2410_02395_amd import mbs
    reqs = make_requests(14, "cuda:0")
    # keep the test quick: only the smaller edges
    reqs = [r for r in reqs if r.shape[0] <= 128][:10]
    assert len(reqs) >= 4
    mix = [copy.copy(r) for r in reqs]
    ser = [copy.copy(r) for r in reqs]
    srv = Server(200e9, slots_for=lambda s: 3, check_every=16)
    done_mix = srv.run(mix, realtime=False)
    # admission respected the budget
    assert srv.used <= srv.budget
    srv.close()
    done_ser = run_serial(ser, realtime=False, check_every=16)
    by_id = {r.id: r for r in done_ser}
    for r in done_mix:
        s = by_id[r.id]
        print(f"req {r.id} {r.shape} it {r.result['iterations']} / {s.result['iterations']} "
              f"eps {r.result['rel_residual']:.2e}", flush=True)
        assert r.result["converged"] == 1 and s.result["converged"] == 1
        assert r.result["iterations"] == s.result["iterations"]
        assert torch.equal(r.out, s.out)
    # equal residual on both sides, re-evaluated by the library
    r = done_mix[0]
    with mbs.Plan(r.shape) as plan:
        plan.set_medium(0, r.n, r.k0, r.ramp_width, r.ramp_max)
        plan.solve(0, r.S, 1e-2, 5)              # sets the slot's source
        rr = plan.residual(0, r.out)
        assert rr < 1.05e-4
    print(summarize(done_mix), summarize(done_ser))


def test_budget_queues_instead_of_overallocating():
    import sys, os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from bench import make_requests
    from paper_2410_02395_amd import mbs
    from paper_2410_02395_amd.serve import Server
    reqs = [r for r in make_requests(14, "cuda:0") if r.shape[0] in (64, 96)][:6]
    assert len({r.shape for r in reqs}) == 2
    # a plan that can never fit is rejected, not left waiting
    none = Server(0.0)
    done = none.run([copy.copy(reqs[0])], realtime=False)
    assert done[0].result["status"] == mbs.MBS_ENOMEM and not none.pools
    # room for one plan at a time: plans are created and evicted in turn, never over budget
    big = max(Server().plan_bytes(r.shape) for r in reqs)
    one = Server(big)
    peak = 0
    orig = one._admit

    def admit(now):
        nonlocal peak
        orig(now)
        peak = max(peak, one.used)

    one._admit = admit
    done = one.run([copy.copy(r) for r in reqs], realtime=False)
    assert peak <= one.budget
    assert len(done) == len(reqs) and all(r.result["converged"] == 1 for r in done)
    one.close()
