"""GPU parity of the batched path (one persistent launch over many uneven
systems) against the oracle, system by system, plus the hipGraph replay and
per-system failure reporting.  Bars as for the single-system loop: iteration
count within +-1 of the oracle, the same stop reason, backward error
<= 1e-14, forward error within the stated bound."""
import sys

import numpy as np
import pytest

from paper_2311_14616_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_14616_amd import mpir
    mpir.lib()
    return mpir


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


SIZES = [1, 2, 31, 32, 33, 63, 64, 65, 100, 257, 300, 511, 512, 513, 1000, 1024]


def _systems(seed=7, count=len(SIZES)):
    ns, alphas, ds = I.batched_spec(count=count, seed=seed)
    ns = np.array(SIZES[:count]) if count <= len(SIZES) else ns
    out = []
    rng = np.random.default_rng(seed)
    for k, n in enumerate(ns):
        at = I.batched_system(int(n), float(rng.uniform(0.5, 5.0)), rng.uniform(0, 0.1, int(n)))
        out.append((int(n), at, I.rhs_ones(at)))
    return out


def _one_config(M, panel, update):
    t = M.Tuning()
    t.nclass = 1
    t.nmax[0] = 1024
    t.panel[0] = panel
    t.update[0] = update
    return t


# every configuration the autotuner can pick: panel width x update form
CONFIGS = [(None, None), (16, 0), (16, 1), (32, 0), (32, 1), (32, 2)]


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: "default" if c[0] is None else f"p{c[0]}u{c[1]}")
@pytest.mark.parametrize("tf", ["f32", "f16", "bf16"])
def test_batched_parity_against_oracle(M, orc, tf, cfg):
    say(f"batched parity tf={tf} cfg={cfg}")
    T = {"f32": M.F32, "f16": M.F16, "bf16": M.BF16}[tf]
    if cfg[0] is not None:
        M.batch_set_tuning(M.F64, T, _one_config(M, *cfg))
    try:
        _parity_run(M, orc, tf)
    finally:
        M.batch_set_tuning(M.F64, T, None)


def _parity_run(M, orc, tf):
    systems = _systems()
    As = [dev(at) for _, at, _ in systems]
    bs = [dev(b) for _, _, b in systems]
    xs = [torch.empty_like(b) for b in bs]
    T = {"f32": M.F32, "f16": M.F16, "bf16": M.BF16}[tf]
    tp = M.term(tol_rel=1e-14, litmax=20)
    bt = M.Batch(As, bs, xs, T, term_parms=tp, use_graph=False)
    st, reps = bt.run()
    bt.destroy()
    assert st == M.OK
    for (n, at, b), x, rep in zip(systems, xs, reps):
        ref = orc.ir_solve(at, b, {"f32": orc.F32, "f16": orc.F16, "bf16": orc.BF16}[tf], tol_rel=1e-14,
                           litmax=20)
        assert rep.reserved == 0 and rep.info == 0
        assert rep.stop_name == ref.stop_name == "converged", (n, rep.stop_name, ref.stop_name)
        assert abs(rep.n_iter - ref.n_iter) <= 1, (n, rep.n_iter, ref.n_iter)
        assert rep.bwd_err <= 1e-14
        assert rep.rhist[0] == ref.rhist[0] and rep.anorm_inf == ref.anorm
        xg = x.cpu().numpy()
        xref, _, _ = orc.solve_f64(at, b)
        kappa = np.abs(at).sum(0).max() * np.abs(np.linalg.inv(at.T)).sum(1).max()
        assert np.abs(xg - xref).max() / np.abs(xref).max() <= 1e-12 * kappa * (2.0**-53 / 1e-16)


def test_batched_extended_residual(M, orc):
    say("batched tw=f32 tr=f64")
    ns = [50, 200, 333]
    sysl = [I.wilkinson_operator(n, 1e5, seed=100 + n) for n in ns]
    As = [dev(s[0]) for s in sysl]
    bs = [dev(s[1]) for s in sysl]
    xs = [torch.empty_like(b) for b in bs]
    bt = M.Batch(As, bs, xs, M.F32, term_parms=M.term(litmax=20), use_graph=False)
    st, reps = bt.run()
    bt.destroy()
    for (at, b, _, _), x, rep in zip(sysl, xs, reps):
        ref = orc.ir_solve(at, b, orc.F32, tr=orc.F64, litmax=20)
        assert rep.stop_name == ref.stop_name
        assert abs(rep.n_iter - ref.n_iter) <= 1
        xp, _, _ = orc.solve_f64(at, b)
        assert np.abs(x.cpu().numpy().astype(np.float64) - xp).max() / np.abs(xp).max() <= 4 * 2.0**-24


@pytest.mark.parametrize("cfg", CONFIGS[1:], ids=lambda c: f"p{c[0]}u{c[1]}")
def test_batched_extended_residual_every_form(M, orc, cfg):
    # TW = F32 with TR = F64 (stop by eq. wilkterm) through every tuned panel
    # width and update form, on sizes that span several panels and pairs
    say(f"batched tw=f32 tr=f64 cfg={cfg}")
    M.batch_set_tuning(M.F32, M.F32, _one_config(M, *cfg))
    try:
        ns = [33, 100, 257, 513, 700]
        sysl = [I.wilkinson_operator(n, 1e4, seed=200 + n) for n in ns]
        As = [dev(s[0]) for s in sysl]
        bs = [dev(s[1]) for s in sysl]
        xs = [torch.empty_like(b) for b in bs]
        bt = M.Batch(As, bs, xs, M.F32, term_parms=M.term(litmax=20), use_graph=False)
        st, reps = bt.run()
        bt.destroy()
        assert st == M.OK
        for (at, b, _, _), x, rep in zip(sysl, xs, reps):
            ref = orc.ir_solve(at, b, orc.F32, tr=orc.F64, litmax=20)
            assert rep.stop_name == ref.stop_name
            assert abs(rep.n_iter - ref.n_iter) <= 1
            xp, _, _ = orc.solve_f64(at, b)
            assert np.abs(x.cpu().numpy().astype(np.float64) - xp).max() / np.abs(xp).max() <= 4 * 2.0**-24
    finally:
        M.batch_set_tuning(M.F32, M.F32, None)


def test_batched_graph_replays_match_eager(M):
    say("batched graph replay")
    systems = _systems(seed=3, count=12)
    As = [dev(at) for _, at, _ in systems]
    bs = [dev(b) for _, _, b in systems]
    tp = M.term(tol_rel=1e-14, litmax=20)
    xe = [torch.empty_like(b) for b in bs]
    eager = M.Batch(As, bs, xe, M.F32, term_parms=tp, use_graph=False)
    st, reps_e = eager.run()
    eager.destroy()
    xg = [torch.full_like(b, 7.0) for b in bs]
    g = M.Batch(As, bs, xg, M.F32, term_parms=tp, use_graph=True)
    scratch = torch.zeros(1 << 20, device=DEV)
    for rep_i in range(3):
        for x in xg:
            x.fill_(float(rep_i) + 3.0)          # eager work between replays
        scratch.add_(1.0)
        torch.cuda.synchronize()
        st, reps_g = g.run()
        assert st == M.OK
        for a, b_, ra, rb in zip(xe, xg, reps_e, reps_g):
            assert torch.equal(a, b_)
            assert ra.n_iter == rb.n_iter and list(ra.rhist[:ra.n_iter + 1]) == list(rb.rhist[:rb.n_iter + 1])
    g.destroy()


def test_batched_phase_times(M):
    # the kernel's per-phase device timers cover each system from its first
    # step to its report: their sum over phases matches the per-system
    # factor + refinement times of the reports
    say("batched phase times")
    systems = _systems(seed=5, count=10)
    As = [dev(at) for _, at, _ in systems]
    bs = [dev(b) for _, _, b in systems]
    xs = [torch.empty_like(b) for b in bs]
    M.batch_phase_times(reset=True)
    assert sum(M.batch_phase_times().values()) == 0.0
    bt = M.Batch(As, bs, xs, M.F32, term_parms=M.term(tol_rel=1e-14, litmax=20), use_graph=False)
    st, reps = bt.run()
    bt.destroy()
    assert st == M.OK
    ph = M.batch_phase_times(reset=True)
    assert set(ph) == set(M.BATCH_PHASES)
    assert all(v >= 0.0 for v in ph.values())
    for k in ("downcast", "panel", "interchanges", "u_rows", "update", "solves", "residual"):
        assert ph[k] > 0.0, k
    tot = sum(ph.values())
    rep_tot = sum(r.t_factor_ms + r.t_ir_ms for r in reps)
    lu = sum(ph[k] for k in ("downcast", "panel", "interchanges", "u_rows", "update"))
    assert abs(tot - rep_tot) <= 0.02 * rep_tot + 1e-3, (tot, rep_tot)
    assert abs(lu - sum(r.t_factor_ms for r in reps)) <= 0.02 * lu + 1e-3
    assert sum(M.batch_phase_times().values()) == 0.0


def test_batched_per_system_failures(M):
    say("batched failures")
    good = I.batched_system(40, 1.0, np.zeros(40))
    sing = good.copy()
    sing[5] = 0.0                        # column 5 of A is zero
    nanm = good.copy()
    nanm[3, 3] = np.nan
    mats = [good, sing, nanm, good]
    As = [dev(a) for a in mats]
    bs = [dev(I.rhs_ones(good)) for _ in mats]
    xs = [torch.empty_like(b) for b in bs]
    bt = M.Batch(As, bs, xs, M.F32, use_graph=False)
    st, reps = bt.run()
    bt.destroy()
    assert [r.reserved for r in reps] == [M.OK, M.ERR_SINGULAR, M.ERR_NONFINITE, M.OK]
    assert reps[1].info == 6
    assert st == M.ERR_SINGULAR


def test_batched_full_workload_sampled(M, orc):
    # the full uneven batch: 4096 systems, N_k in [32, 1024]; checked on a
    # sample against the oracle, and every system must converge
    say("batched full workload")
    ns, alphas, ds = I.batched_spec()
    As, bs, xs = [], [], []
    for n, al, d in zip(ns, alphas, ds):
        at = I.gmat_operator_torch(int(n), float(al), DEV)
        at[torch.arange(int(n)), torch.arange(int(n))] += torch.from_numpy(d).to(DEV)
        As.append(at)
        bs.append(at.sum(0))
        xs.append(torch.empty(int(n), dtype=torch.float64, device=DEV))
    tp = M.term(tol_rel=1e-14, litmax=20)
    bt = M.Batch(As, bs, xs, M.F32, term_parms=tp, use_graph=True)
    st, reps = bt.run()
    bt.destroy()
    assert st == M.OK
    assert all(r.stop == 0 and r.bwd_err <= 1e-14 for r in reps)
    for k in np.random.default_rng(0).choice(len(ns), 8, replace=False):
        at = As[k].cpu().numpy()
        b = bs[k].cpu().numpy()
        ref = orc.ir_solve(at, b, orc.F32, tol_rel=1e-14, litmax=20)
        assert abs(reps[k].n_iter - ref.n_iter) <= 1
        assert np.abs(xs[k].cpu().numpy() - ref.x).max() <= 1e-13


@pytest.mark.parametrize("tf", ["f32", "f16", "bf16"])
def test_autotune_table_and_cache(M, tmp_path, tf):
    """The autotuner returns a valid table (every class measured, a
    candidate chosen), installs it, writes its cache, and a second call with
    the same cache reads the same table back instead of measuring."""
    say(f"autotune tf={tf}")
    T = {"f32": M.F32, "f16": M.F16, "bf16": M.BF16}[tf]
    cache = str(tmp_path / f"tune_{tf}.txt")
    try:
        t1 = M.batch_autotune(M.F64, T, cache)
        d1 = t1.as_dict()
        say(d1)
        assert not d1["from_cache"] and d1["classes"][-1]["nmax"] == 1024
        for c in d1["classes"]:
            assert c["panel"] in (16, 32) and c["update"] in (0, 1, 2) and c["ms"] > 0
            assert c["update"] != 2 or c["panel"] == 32
        assert M.batch_get_tuning(M.F64, T).as_dict()["classes"] == d1["classes"]
        t2 = M.batch_autotune(M.F64, T, cache)
        d2 = t2.as_dict()
        assert d2["from_cache"]
        assert [(c["nmax"], c["panel"], c["update"]) for c in d2["classes"]] == \
            [(c["nmax"], c["panel"], c["update"]) for c in d1["classes"]]
    finally:
        M.batch_set_tuning(M.F64, T, None)
