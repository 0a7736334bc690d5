"""GPU tests of the serving loop (continuous batching of resident trajectories).

A step's arithmetic does not depend on the batch it runs in: every result from the
mix must equal, bitwise, the result of the same steps run alone through rd_step,
and the iteration counts and statuses must agree.  Admission must respect the
device-memory budget, and trajectories opened while others run must be admitted as
memory frees up.
"""
import numpy as np
import pytest

from paper_2305_03945_amd import workloads as wl
from tests.rd_cases import max_abs, oracle_opts, oracle_problem, small_cfg

pytestmark = pytest.mark.gpu

MAX_PUMPS = 20000


@pytest.fixture(scope="module")
def rd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_03945_amd import rd as rdmod
    return rdmod


def dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def request(kind, N, bc, precision, seed, hts):
    cfg = small_cfg(kind, N, bc)
    return dict(cfg=cfg, precision=precision, u0=wl.initial_field(cfg, N=N, seed=seed), hts=list(hts))


def opts_for(rd, cfg, precision):
    return rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], omega=cfg["omega"],
                        precision=precision)


def run_alone(rd, req):
    """The same steps, one rd_step call after another, on a fresh context."""
    ctx = rd.Context(0)
    try:
        p = rd.problem_from_config(req["cfg"])
        o = opts_for(rd, req["cfg"], req["precision"])
        u = dev(req["u0"])
        infos = []
        for ht in req["hts"]:
            u, info = ctx.step(u, ht, p, o)
            infos.append(info)
        return u.cpu().numpy(), infos
    finally:
        ctx.close()


def pump_until(ctx, done, on_round=None):
    for n in range(MAX_PUMPS):
        if done():
            return n
        ctx.pump()
        if on_round is not None:
            on_round(n)
    raise AssertionError("serving did not finish within %d pump rounds" % MAX_PUMPS)


MIX = [
    ("allen_cahn", 64, "periodic", "mixed", 11, (1e-3, 2e-3, 1e-3)),
    ("allen_cahn", 64, "periodic", "mixed", 12, (5e-3, 1e-3)),          # same group as the first
    ("allen_cahn", 128, "neumann", "fp64", 13, (1e-3, 1e-3)),
    ("cahn_hilliard", 64, "neumann", "mixed", 14, (1e-4, 5e-5, 1e-4)),
    ("cahn_hilliard", 32, "periodic", "fp64", 15, (1e-4,)),
    ("schnakenberg", 128, "periodic", "mixed", 16, (1e-3, 2e-3)),
    ("schnakenberg", 64, "neumann", "fp64", 17, (1e-3,)),
]


def test_results_in_the_mix_equal_results_alone(rd):
    reqs = [request(*m) for m in MIX]
    ctx = rd.Context(0)
    try:
        trajs, tickets = [], []
        for r in reqs:
            t = ctx.open(rd.problem_from_config(r["cfg"]), opts_for(rd, r["cfg"], r["precision"]), dev(r["u0"]))
            trajs.append(t)
            tickets.append([t.submit(ht) for ht in r["hts"]])
        infos = {}

        def all_done():
            for tl in tickets:
                for tk in tl:
                    if tk not in infos:
                        i = ctx.poll(tk)
                        if i is not None:
                            infos[tk] = i
            return len(infos) == sum(len(tl) for tl in tickets)

        pump_until(ctx, all_done)
        for r, t, tl in zip(reqs, trajs, tickets):
            alone, alone_infos = run_alone(rd, r)
            mixed = t.read().cpu().numpy()
            assert np.array_equal(mixed, alone), (r["cfg"]["kind"], r["cfg"]["N"], max_abs(mixed, alone))
            for tk, ai in zip(tl, alone_infos):
                si = infos[tk]
                assert (si["iters"], si["outer"], si["status"]) == (ai["iters"], ai["outer"], ai["status"]), (si, ai)
                assert si["residual"] == ai["residual"]
            t.close()
    finally:
        ctx.close()


def test_mixed_serving_result_matches_oracle(rd):
    """One served Allen-Cahn step against the FP64 oracle, at the mixed path's 1e-5."""
    from oracle import pdhg as opdhg
    req = request("allen_cahn", 64, "periodic", "mixed", 21, (1e-3,))
    cfg = req["cfg"]
    ctx = rd.Context(0)
    try:
        t = ctx.open(rd.problem_from_config(cfg), opts_for(rd, cfg, "mixed"), dev(req["u0"]))
        tk = t.submit(req["hts"][0])
        pump_until(ctx, lambda: ctx.poll(tk) is not None)
        got = t.read().cpu().numpy()
        ref = opdhg.step(oracle_problem(cfg), req["u0"], req["hts"][0], oracle_opts(cfg, tol=1e-10))
        assert max_abs(got, ref.U) <= 1e-5
        t.close()
    finally:
        ctx.close()


def test_budget_bounds_admission_and_queued_work_completes(rd):
    """Five trajectories, a budget that holds two workspaces: never more than two
    admitted, and closing finished trajectories lets the queued ones in."""
    reqs = [request("allen_cahn", 128, "periodic", "mixed", 30 + i, (1e-3, 1e-3)) for i in range(5)]
    ctx = rd.Context(0)
    try:
        cfg = reqs[0]["cfg"]
        p = rd.problem_from_config(cfg)
        o = opts_for(rd, cfg, "mixed")
        fp = rd.footprint_bytes(p, o)
        assert fp > 0
        ctx.set_budget(2 * fp)
        trajs = [ctx.open(p, o, dev(r["u0"])) for r in reqs]
        tickets = [[t.submit(ht) for ht in r["hts"]] for t, r in zip(trajs, reqs)]
        results = [None] * len(reqs)
        seen_admitted = []

        def check(_):
            st = ctx.serve_stats()
            assert st["resident_bytes"] <= st["budget_bytes"]
            assert st["admitted"] <= 2
            seen_admitted.append(st["admitted"])
            for i, t in enumerate(trajs):
                if t is not None and all(ctx.poll(tk) is not None for tk in tickets[i]):
                    results[i] = t.read().cpu().numpy()
                    t.close()
                    trajs[i] = None

        pump_until(ctx, lambda: all(r is not None for r in results), on_round=check)
        assert max(seen_admitted) == 2
        st = ctx.serve_stats()
        assert st["admitted"] == 0 and st["queued"] == 0 and st["resident_bytes"] == 0
        for r, res in zip(reqs, results):
            alone, _ = run_alone(rd, r)
            assert np.array_equal(res, alone)
    finally:
        ctx.close()


def test_late_arrivals_join_running_batches(rd):
    """Requests submitted while others are mid-step start at the next round and
    finish with the same result as alone (continuous batching, not a queue)."""
    first = request("allen_cahn", 64, "periodic", "fp64", 41, (1e-3, 1e-3, 1e-3))
    late = [request("allen_cahn", 64, "periodic", "fp64", 42, (2e-3,)),
            request("schnakenberg", 64, "periodic", "mixed", 43, (1e-3,))]
    ctx = rd.Context(0)
    try:
        t0 = ctx.open(rd.problem_from_config(first["cfg"]), opts_for(rd, first["cfg"], "fp64"), dev(first["u0"]))
        tk0 = [t0.submit(ht) for ht in first["hts"]]
        ctx.pump()
        st = ctx.serve_stats()
        assert st["admitted"] == 1 and st["queued"] == 0
        late_t, late_tk = [], []
        for r in late:
            t = ctx.open(rd.problem_from_config(r["cfg"]), opts_for(rd, r["cfg"], r["precision"]), dev(r["u0"]))
            late_t.append(t)
            late_tk.append([t.submit(ht) for ht in r["hts"]])
        ctx.pump()
        st = ctx.serve_stats()
        # the late requests were admitted and started while the first one still had work
        assert st["admitted"] == 3
        assert any(ctx.poll(tk) is None for tk in tk0)
        pump_until(ctx, lambda: all(ctx.poll(tk) is not None for tl in [tk0] + late_tk for tk in tl))
        for r, t in zip([first] + late, [t0] + late_t):
            alone, _ = run_alone(rd, r)
            assert np.array_equal(t.read().cpu().numpy(), alone)
            t.close()
    finally:
        ctx.close()


def test_poll_and_argument_errors(rd):
    ctx = rd.Context(0)
    try:
        with pytest.raises(rd.RDError):
            ctx.poll(123456789)
        with pytest.raises(rd.RDError):
            ctx.pump(-1)
        cfg = small_cfg("allen_cahn", 64, "periodic")
        t = ctx.open(rd.problem_from_config(cfg), opts_for(rd, cfg, "fp64"), dev(wl.initial_field(cfg, N=64)))
        with pytest.raises(rd.RDError):
            t.submit(0.0)
        with pytest.raises(rd.RDError):
            t.submit(float("nan"))
        t.close()
        with pytest.raises(rd.RDError):   # a closed trajectory has no handle left
            t.submit(1e-3)
    finally:
        ctx.close()


def test_trajectory_outliving_its_context(rd):
    """Closing a context frees its trajectories: a trajectory object kept past that point
    refuses to submit or read, and closing it is a no-op (no freed handle reaches the C
    library)."""
    ctx = rd.Context(0)
    cfg = small_cfg("allen_cahn", 64, "periodic")
    t = ctx.open(rd.problem_from_config(cfg), opts_for(rd, cfg, "fp64"), dev(wl.initial_field(cfg, N=64)))
    t.submit(cfg["ht"])
    ctx.close()
    with pytest.raises(rd.RDError):
        t.submit(cfg["ht"])
    with pytest.raises(rd.RDError):
        t.read()
    t.close()
    t.close()


def test_close_drops_queued_steps(rd):
    """Closing a trajectory with steps still queued releases their tickets (polling one
    raises instead of staying busy), and another trajectory's step still completes with
    the result it has alone."""
    ctx = rd.Context(0)
    try:
        cfg = small_cfg("allen_cahn", 64, "periodic")
        p, o = rd.problem_from_config(cfg), opts_for(rd, cfg, "fp64")
        u0 = wl.initial_field(cfg, N=64)
        a = ctx.open(p, o, dev(u0))
        b = ctx.open(p, o, dev(u0))
        ta = [a.submit(cfg["ht"]) for _ in range(3)]
        tb = b.submit(cfg["ht"])
        ctx.pump()
        a.close()
        for tk in ta:
            with pytest.raises(rd.RDError):
                ctx.poll(tk)
        pump_until(ctx, lambda: ctx.poll(tb) is not None)
        alone, info = ctx.step(dev(u0), cfg["ht"], p, o)
        assert ctx.poll(tb)["iters"] == info["iters"]
        assert np.array_equal(b.read().cpu().numpy(), alone.cpu().numpy())
        b.close()
    finally:
        ctx.close()


def test_read_while_a_round_runs(rd):
    """A read issued while the trajectory's round is in flight returns a whole state: the
    initial one or the result of a finished step, each bitwise as computed alone."""
    ctx = rd.Context(0)
    try:
        cfg = small_cfg("allen_cahn", 256, "periodic")
        p, o = rd.problem_from_config(cfg), opts_for(rd, cfg, "fp64")
        u0 = wl.initial_field(cfg, N=256)
        s1, _ = ctx.step(dev(u0), cfg["ht"], p, o)
        s2, _ = ctx.step(s1.clone(), cfg["ht"], p, o)
        whole = [u0, s1.cpu().numpy(), s2.cpu().numpy()]
        t = ctx.open(p, o, dev(u0))
        tickets = [t.submit(cfg["ht"]) for _ in range(2)]
        seen = 0
        for _ in range(MAX_PUMPS):
            if all(ctx.poll(tk) is not None for tk in tickets):
                break
            ctx.pump()
            r = t.read().cpu().numpy()
            k = [i for i, w in enumerate(whole) if np.array_equal(r, w)]
            assert k and k[0] >= seen, "read returned a state that is no step's result"
            seen = k[0]
        assert np.array_equal(t.read().cpu().numpy(), whole[2])
        t.close()
    finally:
        ctx.close()


@pytest.mark.parametrize("N", [64, 256])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_failed_step_leaves_the_state(rd, N, precision):
    """A served step that fails (here: the iteration limit) reports the status rd_step
    reports alone and leaves the trajectory at U^k; a later step with room to converge
    starts from U^k and gives the step's result alone."""
    ctx = rd.Context(0)
    try:
        cfg = small_cfg("allen_cahn", N, "periodic")
        p = rd.problem_from_config(cfg)
        tight = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], max_iter=3, max_outer=1,
                             precision=precision)
        u0 = wl.initial_field(cfg, N=N)
        _, alone = ctx.step(dev(u0), cfg["ht"], p, tight)
        assert alone["status"] != "ok", alone
        t = ctx.open(p, tight, dev(u0))
        tk = t.submit(cfg["ht"])
        pump_until(ctx, lambda: ctx.poll(tk) is not None)
        info = ctx.poll(tk)
        assert (info["status"], info["iters"], info["outer"]) == (alone["status"], alone["iters"], alone["outer"])
        assert np.array_equal(t.read().cpu().numpy(), u0)
        t.close()
        o = opts_for(rd, cfg, precision)
        t = ctx.open(p, o, dev(u0))
        tk = t.submit(cfg["ht"])
        pump_until(ctx, lambda: ctx.poll(tk) is not None)
        ref, ref_info = ctx.step(dev(u0), cfg["ht"], p, o)
        assert ctx.poll(tk)["status"] == ref_info["status"] == "ok"
        assert np.array_equal(t.read().cpu().numpy(), ref.cpu().numpy())
        t.close()
    finally:
        ctx.close()


def test_fch_and_3d_trajectories_in_the_mix(rd):
    """Sixth-order (FP64 and mixed) and 3-D trajectories served beside 2-D ones: each result
    equals its steps run alone through rd_step, bitwise, with the same iteration counts."""
    import math
    fch = rd.make_problem("fch", 64, L=2 * math.pi, diff=(0.18 ** 2,))
    fch_o = rd.make_opts(tol=1e-6, tau_u=0.58, tau_p=0.58, max_iter=5000)
    fch_m = rd.make_opts(tol=1e-6, tau_u=0.58, tau_p=0.58, max_iter=5000, precision="mixed")
    x = np.arange(64) * (2 * math.pi / 64)
    X, Y = np.meshgrid(x, x)
    fch_u0 = 2 * np.exp(np.sin(X) + np.sin(Y) - 2) + 2.2 * np.exp(-np.sin(X) - np.sin(Y) - 2) - 1
    c3 = dict(small_cfg("allen_cahn", 32, "neumann"), dim=3)
    p3 = rd.problem_from_config(c3)
    o3 = opts_for(rd, c3, "mixed")
    u3 = wl.uniform_field(32, -0.5, 0.5, 44, 3)
    c2 = small_cfg("schnakenberg", 64, "periodic")
    jobs = [(fch, fch_o, fch_u0, (1e-3, 1e-3)), (fch, fch_m, fch_u0, (1e-3, 2e-3)), (p3, o3, u3, (1e-3, 2e-3)),
            (rd.problem_from_config(c2), opts_for(rd, c2, "mixed"), wl.initial_field(c2, N=64, seed=45), (1e-3,))]
    alone = []
    actx = rd.Context(0)
    try:
        for p, o, u0, hts in jobs:
            u, infos = dev(u0), []
            for ht in hts:
                u, info = actx.step(u, ht, p, o)
                infos.append(info)
            alone.append((u.cpu().numpy(), infos))
    finally:
        actx.close()
    ctx = rd.Context(0)
    try:
        trajs = [ctx.open(p, o, dev(u0)) for p, o, u0, _ in jobs]
        tickets = [[t.submit(ht) for ht in job[3]] for t, job in zip(trajs, jobs)]
        infos = {}

        def done():
            for tl in tickets:
                for tk in tl:
                    if tk not in infos:
                        i = ctx.poll(tk)
                        if i is not None:
                            infos[tk] = i
            return len(infos) == sum(len(tl) for tl in tickets)

        pump_until(ctx, done)
        for t, tl, (ref, ref_infos) in zip(trajs, tickets, alone):
            assert np.array_equal(t.read().cpu().numpy(), ref)
            for tk, ai in zip(tl, ref_infos):
                assert infos[tk]["status"] == "ok"
                assert (infos[tk]["iters"], infos[tk]["outer"]) == (ai["iters"], ai["outer"])
            t.close()
    finally:
        ctx.close()
