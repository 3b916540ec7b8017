"""Continuous-batching server: results alone vs in the mix, admission, failure isolation."""
import time

import numpy as np
import pytest

from gpu_util import host, model_for, say, torch_cuda
from oracle import solve as osolve
from rte_inputs import configs

pytestmark = pytest.mark.gpu


def _requests(count, grids=(16, 32), ndirs=(16,)):
    return [configs.c3_request(r, ndir_choices=ndirs, grid_choices=grids) for r in range(count)]


def _build(reqs):
    from paper_2604_23265_amd import api
    models = {}
    ops = []
    for p in reqs:
        N = p["dirs"].shape[0]
        if N not in models:
            models[N] = model_for(p)[0]
        ops.append(api.Operator(p, model=models[N]))
    return models, ops


def _wait(srv, tickets, timeout=120.0):
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        for t in tickets:
            if t in done:
                continue
            r = srv.poll(t)
            if r is not None:
                done[t] = r
        assert time.time() - t0 < timeout, "server did not finish in time"
        time.sleep(0.001)
    return done


def test_results_alone_equal_results_in_the_mix():
    torch = torch_cuda()
    from paper_2604_23265_amd import api
    say("case serving mix of 8 requests")
    reqs = _requests(8)
    models, ops = _build(reqs)
    kw = dict(restart=30, rtol=1e-8, precond="bf16")
    alone = []
    for p, op in zip(reqs, ops):
        x, st = op.solve(**kw)
        assert st["converged"] == 1
        alone.append(x.clone())
    srv = api.Server(arena_bytes=512 << 20, max_slots=4)
    outs = [torch.full((op.n,), float("nan"), dtype=torch.float64, device="cuda") for op in ops]
    tickets = [srv.submit(op, out, model=op.model, **kw) for op, out in zip(ops, outs)]
    done = _wait(srv, tickets)
    q = srv.query()
    say("  server", q)
    srv.close()
    for t, a, out, p in zip(tickets, alone, outs, reqs):
        code, st = done[t]
        assert code == 0 and st["converged"] == 1
        assert bool((out == a).all()), "result differs between alone and in the mix"
    assert q["completed"] == len(reqs) and q["arena_peak"] <= q["arena_bytes"]
    # and the served results satisfy the FP64 residual check of the oracle
    P = osolve.Problem(reqs[0])
    assert osolve.relative_residual(P, host(outs[0])) <= 1e-8 * 1.01


def _shape_requests():
    import problems
    reqs = []
    for s in range(3):  # 3D, 32 directions, 48-channel MgNet: the tiled 3D convolutions
        reqs.append(problems.make(dim=3, n=8, ndir=32, g=0.6, eps=0.2, kind="sphere", inflow="random",
                                  seed=40 + s, mg=dict(c0=48, levels=2, nu_pre=2, nu_post=2, nu_coarse=2,
                                                       coef_ch=3, seed=7)))
    for s in range(3):  # 2D, 64 directions: the matrix-core apply
        reqs.append(problems.make(n=16, ndir=64, g=0.8, eps=0.1, inflow="random", seed=50 + s,
                                  mg=dict(c0=32, levels=2, nu_pre=2, nu_post=2, nu_coarse=2, coef_ch=3, seed=8)))
    for s in range(2):  # 3D, 96 directions: both
        reqs.append(problems.make(dim=3, n=4, ndir=96, g=0.8, eps=0.3, kind="sphere", inflow="random",
                                  seed=60 + s, mg=dict(c0=96, levels=2, nu_pre=2, nu_post=2, nu_coarse=2,
                                                       coef_ch=3, seed=9)))
    return reqs


def test_results_alone_equal_results_in_the_mix_3d_and_wide_angle_shapes():
    """Batches of 3D and 64/96-direction solves (every launch covering 2 or 3 solves) give
    each solve the same bits as alone."""
    torch = torch_cuda()
    from paper_2604_23265_amd import api
    say("case serving mix of 3D and wide-angle shapes")
    reqs = _shape_requests()
    models, ops = _build(reqs)
    kw = dict(restart=30, rtol=1e-8, precond="bf16", max_iters=3000)
    alone = []
    for op in ops:
        x, st = op.solve(**kw)
        assert st["converged"] == 1, st
        alone.append(x.clone())
    srv = api.Server(arena_bytes=512 << 20, max_slots=4)
    outs = [torch.full((op.n,), float("nan"), dtype=torch.float64, device="cuda") for op in ops]
    tickets = [srv.submit(op, out, model=op.model, **kw) for op, out in zip(ops, outs)]
    done = _wait(srv, tickets)
    srv.close()
    for t, a, out in zip(tickets, alone, outs):
        code, st = done[t]
        assert code == 0 and st["converged"] == 1
        assert bool((out == a).all()), "result differs between alone and in the mix"
    for i in (0, 3, 6):
        assert osolve.relative_residual(osolve.Problem(reqs[i]), host(outs[i])) <= 1e-8 * 1.01


def test_fp64_residual_kernels_agree_bitwise_in_the_server():
    """The server's restart residuals on the FP64 matrix cores (16, 32, 64 and 96 directions,
    2D and 3D) against the vector kernel (RTE_APPLY64_VEC=1): the two agree bit for bit, so a
    served batch takes the same iterations and restarts and returns the same bits.  Both runs
    are eager (RTE_GRAPHS=0) so that each launch reads the switch."""
    import os
    torch = torch_cuda()
    from paper_2604_23265_amd import api
    say("case served batch, matrix-core vs vector FP64 residual")
    reqs = _requests(4, grids=(16, 32), ndirs=(16, 32)) + _shape_requests()[2:5] + _shape_requests()[6:7]
    models = [model_for(p)[0] for p in reqs]  # one per request: 2D and 3D share direction counts
    ops = [api.Operator(p, model=m) for p, m in zip(reqs, models)]
    kw = dict(restart=10, rtol=1e-8, precond="bf16", max_iters=3000)
    runs = {}
    os.environ["RTE_GRAPHS"] = "0"
    try:
        for vec in ("1", "0"):
            os.environ["RTE_APPLY64_VEC"] = vec
            srv = api.Server(arena_bytes=512 << 20, max_slots=4)
            outs = [torch.full((op.n,), float("nan"), dtype=torch.float64, device="cuda") for op in ops]
            tickets = [srv.submit(op, out, model=op.model, **kw) for op, out in zip(ops, outs)]
            done = _wait(srv, tickets)
            srv.close()
            runs[vec] = (outs, [done[t] for t in tickets])
    finally:
        os.environ.pop("RTE_APPLY64_VEC", None)
        os.environ.pop("RTE_GRAPHS", None)
    for (ov, (cv, sv)), (om, (cm, sm)) in zip(zip(runs["1"][0], runs["1"][1]), zip(runs["0"][0], runs["0"][1])):
        assert cv == 0 and cm == 0 and sv["converged"] == 1 and sm["converged"] == 1
        assert sv["iterations"] == sm["iterations"] and sv["restarts"] == sm["restarts"]
        assert bool((ov == om).all()), "served results differ between the residual kernels"
    say("  iterations", [st["iterations"] for _, st in runs["0"][1]])


def test_admission_by_footprint():
    torch = torch_cuda()
    from paper_2604_23265_amd import api
    say("case serving admission")
    reqs = _requests(6, grids=(32,))
    models, ops = _build(reqs)
    kw = dict(restart=20, rtol=1e-6, precond="bf16")
    need = ops[0].workspace_bytes(ops[0].model, **kw)
    srv = api.Server(arena_bytes=int(2.5 * need) + 4096, max_slots=8)   # room for two at a time
    outs = [torch.empty(op.n, dtype=torch.float64, device="cuda") for op in ops]
    tickets = [srv.submit(op, out, model=op.model, **kw) for op, out in zip(ops, outs)]
    done = _wait(srv, tickets)
    q = srv.query()
    srv.close()
    assert all(done[t][0] == 0 for t in tickets)
    assert q["arena_peak"] <= q["arena_bytes"] and q["arena_peak"] >= need
    assert q["arena_peak"] < 3 * need


def test_errors_and_poisoned_request_isolation():
    torch = torch_cuda()
    from paper_2604_23265_amd import _lib as L
    from paper_2604_23265_amd import api
    say("case serving errors")
    reqs = _requests(3)
    models, ops = _build(reqs)
    kw = dict(restart=30, rtol=1e-8, precond="fp32")
    small = api.Server(arena_bytes=1 << 20, max_slots=2)
    with pytest.raises(L.RteError) as e:
        small.submit(ops[0], torch.empty(ops[0].n, dtype=torch.float64, device="cuda"), model=ops[0].model, **kw)
    assert e.value.code == L.RTE_ENOMEM
    with pytest.raises(L.RteError) as e:
        small.poll(12345)
    assert e.value.code == L.RTE_ENOTFOUND
    small.close()

    srv = api.Server(arena_bytes=256 << 20, max_slots=3)
    bad_b = torch.full((ops[1].n,), float("nan"), dtype=torch.float64, device="cuda")
    outs = [torch.empty(op.n, dtype=torch.float64, device="cuda") for op in ops]
    t0 = srv.submit(ops[0], outs[0], model=ops[0].model, **kw)
    t1 = srv.submit(ops[1], outs[1], model=ops[1].model, b=bad_b, **kw)
    t2 = srv.submit(ops[2], outs[2], model=ops[2].model, **kw)
    done = _wait(srv, [t0, t1, t2])
    srv.close()
    assert done[t1][0] in (L.RTE_EINVAL, L.RTE_EBREAKDOWN)
    for t, op, out in ((t0, ops[0], outs[0]), (t2, ops[2], outs[2])):
        assert done[t][0] == 0
        x, st = op.solve(**kw)
        assert bool((x == out).all())


def test_staggered_joins_and_per_slot_restarts():
    """Solves that join a running batch at different steps, restart at different
    steps (short cycles) and reuse freed slots give the results, iteration and
    restart counts they give alone; the iteration limit and a zero right-hand
    side end a solve inside the mix."""
    torch = torch_cuda()
    from paper_2604_23265_amd import _lib as L
    from paper_2604_23265_amd import api
    say("case serving staggered joins, restart 5")
    reqs = [configs.c3_request(r, ndir_choices=(16,), grid_choices=(32,)) for r in range(100, 107)]
    models, ops = _build(reqs)
    kw = [dict(restart=5, rtol=1e-8, precond="bf16") for _ in ops]
    kw[3]["max_iters"] = 7
    zero_b = torch.zeros(ops[5].n, dtype=torch.float64, device="cuda")
    kw[5]["b"] = zero_b
    alone = []
    for op, k in zip(ops, kw):
        x, st = op.solve(**k)
        alone.append((x.clone(), st))
    assert alone[3][1]["status"] == L.RTE_ENOCONV and alone[3][1]["iterations"] == 7
    assert alone[5][1]["converged"] == 1 and alone[5][1]["iterations"] == 0
    srv = api.Server(arena_bytes=512 << 20, max_slots=3)
    outs = [torch.full((op.n,), float("nan"), dtype=torch.float64, device="cuda") for op in ops]
    tickets = []
    for i, (op, out, k) in enumerate(zip(ops, outs, kw)):
        tickets.append(srv.submit(op, out, model=op.model, **k))
        time.sleep(0.002 * (i % 3))
    done = _wait(srv, tickets)
    srv.close()
    for i, (t, (a, sa), out) in enumerate(zip(tickets, alone, outs)):
        code, st = done[t]
        assert code == sa["status"], i
        assert (st["iterations"], st["restarts"]) == (sa["iterations"], sa["restarts"]), i
        assert bool((out == a).all()), "result %d differs between alone and in the mix" % i
    assert bool((outs[5] == 0).all())


def test_submit_many_burst():
    """A burst queued with one call is admitted together; results equal the
    solves alone, and a burst with an invalid request queues nothing."""
    torch = torch_cuda()
    from paper_2604_23265_amd import _lib as L
    from paper_2604_23265_amd import api
    say("case serving submit_many")
    reqs = [configs.c3_request(r, ndir_choices=(16,), grid_choices=(32,)) for r in range(200, 206)]
    models, ops = _build(reqs)
    kw = dict(restart=30, rtol=1e-8, precond="bf16")
    alone = [op.solve(**kw)[0].clone() for op in ops]
    srv = api.Server(arena_bytes=512 << 20, max_slots=8)
    outs = [torch.full((op.n,), float("nan"), dtype=torch.float64, device="cuda") for op in ops]
    bad = [(ops[0], outs[0], ops[0].model, dict(kw, restart=0))] + [
        (op, out, op.model, kw) for op, out in zip(ops[1:], outs[1:])]
    with pytest.raises(L.RteError) as e:
        srv.submit_many(bad)
    assert e.value.code == L.RTE_EINVAL and srv.query()["submitted"] == 0
    tickets = srv.submit_many([(op, out, op.model, kw) for op, out in zip(ops, outs)])
    done = _wait(srv, tickets)
    srv.close()
    for t, a, out in zip(tickets, alone, outs):
        assert done[t][0] == 0
        assert bool((out == a).all())


def test_operator_freed_while_its_batch_serves_others():
    """A batch is created from the first request's operator; that operator may be
    freed once its ticket is polled, and the requests of the same shape still queued
    behind it must solve exactly as they do alone."""
    torch = torch_cuda()
    from paper_2604_23265_amd import api
    say("case serving: first operator freed after its poll")
    reqs = [configs.c3_request(r, ndir_choices=(16,), grid_choices=(32,)) for r in range(300, 304)]
    models, ops = _build(reqs)
    kw = dict(restart=10, rtol=1e-8, precond="bf16")
    alone = [op.solve(**kw)[0].clone() for op in ops]
    srv = api.Server(arena_bytes=256 << 20, max_slots=1)   # one slot: the others wait in line
    outs = [torch.full((op.n,), float("nan"), dtype=torch.float64, device="cuda") for op in ops]
    tickets = [srv.submit(op, out, model=op.model, **kw) for op, out in zip(ops, outs)]
    first = _wait(srv, tickets[:1])
    assert first[tickets[0]][0] == 0
    ops[0].close()                       # the operator the batch was created from
    ops[0] = None
    torch.cuda.synchronize()
    junk = torch.full((1 << 22,), float("nan"), dtype=torch.float64, device="cuda")  # reuse its memory
    done = _wait(srv, tickets[1:])
    srv.close()
    del junk
    for t, a, out in zip(tickets[1:], alone[1:], outs[1:]):
        assert done[t][0] == 0
        assert bool((out == a).all()), "a request served after the first operator was freed differs"
    assert bool((outs[0] == alone[0]).all())


def test_stream_slice_alone_equals_mix_at_full_sizes():
    """Twelve requests of the serving stream itself (grids 64^2..256^2, 16 and 32 directions,
    log-uniform eps, trained weights per direction count) solved alone through rte_solve and
    then through the server with staggered arrivals at 8 slots: every result, iteration and
    restart count must be bitwise the same, and the FP64 residual the oracle computes for a
    served result must meet the tolerance."""
    import os
    torch = torch_cuda()
    from paper_2604_23265_amd import api
    reqs = [configs.c3_request(r) for r in range(12)]
    say("case stream slice:", [(p["n"][0], p["dirs"].shape[0]) for p in reqs])
    wdir = os.path.join(os.path.dirname(api.__file__), "weights")
    models = {N: api.Model(open(os.path.join(wdir, "c3_n%d.mgn1" % N), "rb").read()) for N in (16, 32)}
    ops = [api.Operator(p, model=models[p["dirs"].shape[0]]) for p in reqs]
    kw = dict(restart=30, rtol=1e-6, max_iters=3000, precond="bf16")
    alone, stats = [], []
    for op in ops:
        x, st = op.solve(model=op.model, **kw)
        alone.append(x.clone())
        stats.append(st)
    say("  alone iterations", [s["iterations"] for s in stats])
    srv = api.Server(arena_bytes=4 << 30, max_slots=8)
    outs = [torch.full((op.n,), float("nan"), dtype=torch.float64, device="cuda") for op in ops]
    tickets = [srv.submit(op, out, model=op.model, **kw) for op, out in zip(ops[:7], outs[:7])]
    time.sleep(0.02)
    tickets += [srv.submit(op, out, model=op.model, **kw) for op, out in zip(ops[7:], outs[7:])]
    done = _wait(srv, tickets, timeout=300.0)
    srv.close()
    for i, t in enumerate(tickets):
        code, st = done[t]
        assert code == stats[i]["status"]
        assert st["iterations"] == stats[i]["iterations"] and st["restarts"] == stats[i]["restarts"]
        assert bool((outs[i] == alone[i]).all()), "request %d differs between alone and in the mix" % i
    P = osolve.Problem(reqs[0])
    res = osolve.relative_residual(P, host(outs[0]))
    say("  oracle FP64 residual of request 0:", res)
    assert stats[0]["converged"] == 1 and res <= 1e-6 * 1.001
