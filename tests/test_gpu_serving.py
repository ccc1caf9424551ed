"""GPU tests of the batched forms of the solver through the C ABI: the
warm-started regularisation path (cggm_solve_path) and the continuous-batching
request server (cggm_server_*).

Bars: a path point is bit-for-bit the solve warm-started from the previous
point; path points reach the oracle's optimum at their penalties (objective
within 1e-8 relative, identical supports outside the borderline band); every
request served in a mix of concurrent requests gives bit-for-bit the result
it gives alone; admission never holds more pool memory than the pool has.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

F_RTOL = 1e-8
SUPPORT_EPS = 1e-6


@pytest.fixture(scope="module")
def cg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1509_04681_amd as m
    m.load()
    return m


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def support_mismatches(G, O):
    G, O = np.abs(np.asarray(G)), np.abs(np.asarray(O))
    border = ((G >= 1e-7) & (G <= 1e-5)) | ((O >= 1e-7) & (O <= 1e-5))
    return int((((G > SUPPORT_EPS) != (O > SUPPORT_EPS)) & ~border).sum())


def test_path_point_is_the_warm_started_solve(cg):
    import torch
    pr = synth.stream_problem(3, p_range=(150, 150), q_range=(130, 130), n_range=(300, 300))
    lL, lT = synth.penalty_path(pr.X, pr.Y, points=5, ratio=0.1)
    X, Y = dev(pr.X), dev(pr.Y)
    print(f"path {pr.name}: lamL {lL[0]:.3g}..{lL[-1]:.3g}", flush=True)
    path = cg.cggm_solve_path(X, Y, lL, lT, tol=1e-7)
    assert len(path) == 5
    prev_L = prev_T = None
    for k in range(5):
        r = cg.cggm_solve(X, Y, lL[k], lT[k], tol=1e-7, warm_Lambda=prev_L, warm_Theta=prev_T)
        print(f"  point {k}: f={path[k].f!r} iters={path[k].iters} status={path[k].status}",
              flush=True)
        assert r.f == path[k].f and r.iters == path[k].iters and r.status == path[k].status
        assert torch.equal(r.Lambda, path[k].Lambda) and torch.equal(r.Theta, path[k].Theta)
        assert [t["f"] for t in r.trace] == [t["f"] for t in path[k].trace]
        prev_L, prev_T = r.Lambda, r.Theta
    # the first point is past the largest penalties: Theta = 0, Lambda diagonal
    assert not path[0].Theta.any()
    L0 = path[0].Lambda.cpu().numpy()
    assert np.count_nonzero(L0 - np.diag(np.diag(L0))) == 0


def test_path_points_reach_the_oracle_optimum(cg):
    import oracle
    oracle.build()
    pr = synth.stream_problem(5, p_range=(40, 40), q_range=(30, 30), n_range=(120, 120))
    lL, lT = synth.penalty_path(pr.X, pr.Y, points=4, ratio=0.05)
    path = cg.cggm_solve_path(dev(pr.X), dev(pr.Y), lL, lT, tol=0.0, max_iter=3000)
    for k in range(4):
        o = oracle.solve(pr.X, pr.Y, lL[k], lT[k], tol=0.0, max_iter=5000, stall_iters=3,
                         lambda_passes=3)
        mL = support_mismatches(path[k].Lambda.cpu().numpy(), o.Lambda)
        mT = support_mismatches(path[k].Theta.cpu().numpy(), o.Theta)
        print(f"point {k}: f_gpu={path[k].f!r} f_oracle={o.f!r} "
              f"rel={abs(path[k].f - o.f) / abs(o.f):.2e} mismatches {mL}/{mT}", flush=True)
        assert abs(path[k].f - o.f) <= F_RTOL * abs(o.f)
        assert mL == 0 and mT == 0


def stream(count, seed0, p_range, q_range, n_range):
    out = []
    for k in range(count):
        pr = synth.stream_problem(seed0 + k, p_range=p_range, q_range=q_range, n_range=n_range)
        lL, lT = synth.penalty_path(pr.X, pr.Y, points=4, ratio=0.2)
        out.append((pr, lL, lT))
    return out


def serve(cg, reqs, slots, pool_bytes, precisions, max_bypass=8):
    import torch
    outs, infos = [], []
    inputs = []
    for pr, lL, lT in reqs:                      # inputs resident before the first submit
        inputs.append((dev(pr.X), dev(pr.Y)))
        outs.append((torch.empty((len(lL), pr.q, pr.q), dtype=torch.float64, device="cuda:0"),
                     torch.empty((len(lL), pr.p, pr.q), dtype=torch.float64, device="cuda:0")))
    torch.cuda.synchronize()
    with cg.Server(slots=slots, pool_bytes=pool_bytes, max_bypass=max_bypass) as srv:
        tickets = []
        for (pr, lL, lT), (X, Y), (Lo, To), prec in zip(reqs, inputs, outs, precisions):
            tickets.append(srv.submit(X, Y, lL, lT, tol=1e-7, precision=prec, max_iter=400,
                                      mixed_min_q=0, Lambda_out=Lo, Theta_out=To))
        for t in tickets:
            infos.append(srv.wait(t))
        st = srv.stats()
    return outs, infos, st


def test_served_results_equal_results_alone(cg):
    import torch
    reqs = stream(10, 100, (60, 400), (60, 400), (200, 600))
    prec = ["fp64", "mixed"] * 5          # mixed forced at these sizes (mixed_min_q = 0)
    print("requests:", [r[0].name for r in reqs], flush=True)
    mix, infos, st = serve(cg, reqs, slots=4, pool_bytes=2 << 30, precisions=prec)
    print(f"mix stats {st}", flush=True)
    assert st["completed"] == 10 and st["peak_bytes_in_use"] <= st["pool_bytes"]
    assert st["max_running"] >= 2                      # requests did overlap
    for k, ((pr, lL, lT), info) in enumerate(zip(reqs, infos)):
        assert info["status"] in (cg.CGGM_OK, cg.CGGM_MAXITER, cg.CGGM_STALLED), info
        # alone: one request on a one-slot server
        alone, ainfo, _ = serve(cg, [(pr, lL, lT)], slots=1, pool_bytes=1 << 30,
                                precisions=[prec[k]])
        print(f"{pr.name} {prec[k]}: f mix={info['f']} alone={ainfo[0]['f']} "
              f"iters={info['iters']}", flush=True)
        assert info["f"] == ainfo[0]["f"] and info["iters"] == ainfo[0]["iters"]
        assert torch.equal(mix[k][0], alone[0][0]) and torch.equal(mix[k][1], alone[0][1])
        # and the one-request server equals the path entry point
        if k < 3:
            path = cg.cggm_solve_path(dev(pr.X), dev(pr.Y), lL, lT, tol=1e-7, max_iter=400,
                                      precision=prec[k], mixed_min_q=0)
            assert [r.f for r in path] == info["f"]
            assert all(torch.equal(r.Lambda, mix[k][0][j]) for j, r in enumerate(path))


def test_admission_is_bounded_by_the_pool(cg):
    reqs = stream(6, 200, (200, 300), (200, 300), (200, 400))
    fps = [cg.cggm_workspace_bytes(pr.n, pr.p, pr.q) for pr, _, _ in reqs]
    pool = int(2.2 * max(fps))                  # room for two or three requests
    small = np.cumsum(sorted(fps))
    most = int((small <= pool).sum())           # most requests that fit at once
    _, infos, st = serve(cg, reqs, slots=6, pool_bytes=pool, precisions=["fp64"] * 6)
    print(f"footprints {fps} pool {pool} stats {st}", flush=True)
    assert st["completed"] == 6 and all(i["status"] in (cg.CGGM_OK, cg.CGGM_STALLED)
                                        for i in infos)
    assert st["peak_bytes_in_use"] <= pool and st["max_running"] <= most
    # intervals on the device never hold more than the pool
    events = sorted([(i["t_admit_ms"], i["footprint"]) for i in infos] +
                    [(i["t_done_ms"], -i["footprint"]) for i in infos],
                    key=lambda e: (e[0], e[1]))
    held = 0
    for _, b in events:
        held += b
        assert held <= pool


def test_server_rejects_and_survives_bad_requests(cg):
    pr = synth.stream_problem(7, p_range=(80, 80), q_range=(70, 70), n_range=(150, 150))
    lL, lT = synth.penalty_path(pr.X, pr.Y, points=2, ratio=0.5)
    X, Y = dev(pr.X), dev(pr.Y)
    fp = cg.cggm_workspace_bytes(pr.n, pr.p, pr.q)
    with cg.Server(slots=2, pool_bytes=fp + 4096) as srv:
        big = synth.stream_problem(8, p_range=(300, 300), q_range=(300, 300), n_range=(150, 150))
        with pytest.raises(cg.CggmError) as e:
            srv.submit(dev(big.X), dev(big.Y), [0.1], [0.1])
        assert e.value.code == cg.CGGM_ECAPACITY
        with pytest.raises(cg.CggmError) as e:
            srv.submit(X, Y, [-1.0], [0.1])
        assert e.value.code == cg.CGGM_EINVAL
        Xbad = X.clone()
        Xbad[3, 5] = float("nan")
        tb = srv.submit(Xbad, Y, lL, lT, tol=1e-6)
        tg = srv.submit(X, Y, lL, lT, tol=1e-6)
        with pytest.raises(cg.CggmError) as e:
            srv.wait(tb)
        assert e.value.code == cg.CGGM_EINVAL
        good = srv.wait(tg)
        assert good["status"] in (cg.CGGM_OK, cg.CGGM_STALLED)
        ref = cg.cggm_solve_path(X, Y, lL, lT, tol=1e-6)
        assert good["f"] == [r.f for r in ref]
        st = srv.stats()
        assert st["rejected"] == 1 and st["completed"] == 2
