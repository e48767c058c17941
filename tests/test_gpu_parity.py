"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

FP64 runs match the oracle to 1e-12 relative L2 at equal iteration count
(messages, means, variances); FP32 runs to 1e-5; converged means match the
sparse direct solve to 1e-5.
"""
import os

import numpy as np
import pytest

from conftest import plane_slot_map
from paper_2404_12968_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_12968_amd import gabp
    return gabp


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def gpu_state(G, ctx):
    mean, var = G.gabp_posterior(ctx)
    prec, info = G.gabp_get_messages(ctx)
    torch.cuda.synchronize()
    return (mean.cpu().numpy().ravel(), var.cpu().numpy().ravel(),
            prec.cpu().double().numpy(), info.cpu().double().numpy())


def compare(prob, og, st, tol):
    """Element-by-element comparison of a GPU state with the oracle's."""
    mu_g, var_g, prec_g, info_g = st
    mu_o, var_o = og.posterior()
    d, y, x, e = plane_slot_map(prob, og.g)
    lam_g = prec_g[d, y, x]
    th_g = info_g[d, y, x]
    errs = {"mu": rel_l2(mu_g, mu_o), "var": rel_l2(var_g, var_o),
            "lam": rel_l2(lam_g, og.lam[e]), "th": rel_l2(th_g, og.th[e])}
    # slots without a sender must be exactly zero
    mask = np.ones(prec_g.shape, dtype=bool)
    mask[d, y, x] = False
    assert np.all(prec_g[mask] == 0) and np.all(info_g[mask] == 0)
    for k, v in errs.items():
        assert v <= tol, (k, v, errs)
    return errs


FP64_CASES = [
    # nx, ny, alpha, bcx, bcy, c, eta, kappa, frac
    (64, 64, 1, I.BC_NEUMANN, I.BC_NEUMANN, 1.0, 0.5, 0.2, 0.05),
    (70, 13, 2, I.BC_NEUMANN, I.BC_NEUMANN, 10.0, 0.5, 0.1, 0.1),
    (130, 9, 2, I.BC_PERIODIC, I.BC_NEUMANN, 10.0, 0.6, 0.05, 0.08),
    (33, 37, 2, I.BC_DIRICHLET, I.BC_PERIODIC, -2.0, 0.6, 0.2, 0.1),
    (45, 20, 1, I.BC_PERIODIC, I.BC_PERIODIC, 1.0, 1.0, 0.3, 0.1),
    (1, 50, 2, I.BC_NEUMANN, I.BC_NEUMANN, 10.0, 0.5, 0.2, 0.2),
    (77, 1, 1, I.BC_NEUMANN, I.BC_DIRICHLET, 1.0, 0.7, 0.2, 0.2),
    (5, 5, 2, I.BC_PERIODIC, I.BC_PERIODIC, 20.0, 0.5, 0.4, 0.3),
    (66, 70, 2, I.BC_NEUMANN, I.BC_DIRICHLET, 10.0, 0.5, 0.05, 0.05),
]


@pytest.mark.parametrize("case", FP64_CASES, ids=lambda c: f"{c[0]}x{c[1]}a{c[2]}bc{c[3]}{c[4]}")
def test_fp64_matches_oracle_at_equal_t(G, oracle_mod, case):
    nx, ny, alpha, bcx, bcy, c, eta, kappa, frac = case
    prob = I.small_lattice(nx, ny, alpha, bc_x=bcx, bc_y=bcy, kappa=kappa, c=c, frac=frac,
                           sigma=0.1, seed=nx * 1000 + ny, dtype="f64", hx=1.0, hy=1.3)
    ctx = G.gabp_create_problem(prob)
    og = oracle_mod.OracleGaBP.from_problem(prob)
    t = 0
    for t_next in (1, 2, 7, 60):
        G.gabp_iterate(ctx, t_next - t, eta)
        og.iterate(t_next - t, eta)
        t = t_next
        compare(prob, og, gpu_state(G, ctx), 1e-12)
    assert G.gabp_iteration_count(ctx) == (60, G.GABP_OK)


def test_parity64_workload_fp64(G, oracle_mod):
    """The 64x64 FP64 workload: equal-t parity, then convergence to 1e-10."""
    prob = I.parity64()
    ctx = G.gabp_create_problem(prob)
    og = oracle_mod.OracleGaBP.from_problem(prob)
    G.gabp_iterate(ctx, 100, prob.damping)
    og.iterate(100, prob.damping)
    compare(prob, og, gpu_state(G, ctx), 1e-12)
    st, it, rel = G.gabp_solve(ctx, 100000, prob.damping, prob.rel_tol, prob.check_every)
    ost, orel = og.solve(100000, prob.damping, prob.rel_tol, prob.check_every)
    assert st == G.GABP_OK and ost == 0
    assert it == og.t
    assert rel <= 1e-10 and abs(rel - orel) <= 1e-12 * max(1.0, orel) + 1e-14
    compare(prob, og, gpu_state(G, ctx), 1e-12)
    A, b = oracle_mod.posterior_system(prob)
    exact = oracle_mod.direct_solve(A, b)
    mu, _ = G.gabp_posterior(ctx, want_var=False)
    assert rel_l2(mu.cpu().numpy(), exact) <= 1e-5


@pytest.mark.parametrize("alpha,bcx,bcy,c", [(1, I.BC_NEUMANN, I.BC_PERIODIC, 1.0),
                                            (2, I.BC_PERIODIC, I.BC_NEUMANN, 10.0),
                                            (2, I.BC_NEUMANN, I.BC_NEUMANN, -2.0)])
def test_fp64_converged_mean_equals_direct_solve(G, oracle_mod, alpha, bcx, bcy, c):
    prob = I.small_lattice(48, 40, alpha, bc_x=bcx, bc_y=bcy, kappa=0.3, c=c, frac=0.1,
                           sigma=0.05, seed=99, dtype="f64")
    ctx = G.gabp_create_problem(prob)
    st, it, rel = G.gabp_solve(ctx, 400000, 0.5, 1e-10, 50)
    assert st == G.GABP_OK, (st, it, rel)
    A, b = oracle_mod.posterior_system(prob)
    exact = oracle_mod.direct_solve(A, b)
    mu, _ = G.gabp_posterior(ctx, want_var=False)
    assert rel_l2(mu.cpu().numpy(), exact) <= 1e-5


@pytest.mark.parametrize("nx,ny,alpha,bcx,bcy", [
    (200, 40, 1, I.BC_NEUMANN, I.BC_NEUMANN),
    (200, 40, 2, I.BC_PERIODIC, I.BC_NEUMANN),
    (300, 24, 2, I.BC_NEUMANN, I.BC_DIRICHLET),
    (261, 17, 2, I.BC_DIRICHLET, I.BC_PERIODIC),
    (133, 13, 2, I.BC_PERIODIC, I.BC_PERIODIC),
])
def test_residual_matches_the_oracle_system(G, oracle_mod, nx, ny, alpha, bcx, bcy):
    """gabp_residual against |A mu - b| / |b| with the oracle's own assembled
    A and b (sparse product of the 1-D Laplacians) and the GPU's FP64 mean, on
    lattices wide enough for tiles whose stencil stays inside (the residual
    kernel evaluates the prior there from per-direction constants) as well as
    boundary tiles."""
    prob = I.small_lattice(nx, ny, alpha, bc_x=bcx, bc_y=bcy, kappa=0.2, frac=0.1, sigma=0.1,
                           seed=nx + 7 * ny, dtype="f64", hx=1.0, hy=1.3)
    ctx = G.gabp_create_problem(prob)
    G.gabp_iterate(ctx, 30, 0.5)
    rel, ab = G.gabp_residual(ctx)
    mu, _ = G.gabp_posterior(ctx, want_var=False)
    A, b = oracle_mod.posterior_system(prob)
    r = A @ mu.cpu().numpy().ravel() - b
    want_abs = np.linalg.norm(r)
    want_rel = want_abs / np.linalg.norm(b)
    assert want_rel > 1e-4          # a residual far from zero: every term matters
    assert ab == pytest.approx(want_abs, rel=1e-11)
    assert rel == pytest.approx(want_rel, rel=1e-11)


@pytest.mark.parametrize("dtype,alpha,nx,ny,bcx,bcy", [
    ("f32", 2, 200, 60, I.BC_NEUMANN, I.BC_NEUMANN),
    ("f32", 2, 261, 53, I.BC_PERIODIC, I.BC_DIRICHLET),
    ("f32", 2, 70, 37, I.BC_DIRICHLET, I.BC_PERIODIC),
    ("f32", 2, 9, 9, I.BC_PERIODIC, I.BC_PERIODIC),
    ("f32", 1, 150, 45, I.BC_NEUMANN, I.BC_PERIODIC),
    ("f64", 2, 140, 40, I.BC_NEUMANN, I.BC_DIRICHLET),
    ("f64", 1, 120, 30, I.BC_PERIODIC, I.BC_NEUMANN),
])
def test_frozen_check_matches_the_oracle_system(G, oracle_mod, dtype, alpha, nx, ny, bcx, bcy):
    """The check once the precision messages froze (means from the frozen
    belief precisions, then the windowed residual): gabp_residual against
    |A mu - b| / |b| with the oracle's assembled A and b and the GPU's FP64
    mean, on lattices with interior tiles, ragged and wrapped tiles, and a
    periodic lattice narrower than the residual's window."""
    if (dtype, alpha) == ("f64", 1):
        prob = I.small_lattice(nx, ny, alpha, bc_x=bcx, bc_y=bcy, kappa=0.1, tracks=5, run=4,
                               sigma=0.05, seed=77, dtype=dtype)
    else:
        prob = I.small_lattice(nx, ny, alpha, bc_x=bcx, bc_y=bcy, kappa=0.12, frac=0.08,
                               sigma=0.05, seed=nx + ny, dtype=dtype)
    ctx = G.gabp_create_problem(prob)
    assert _freeze(G, ctx) > 0
    G.gabp_iterate(ctx, 3, 0.5)
    rel, ab = G.gabp_residual(ctx)
    mu, _ = G.gabp_posterior(ctx, want_var=False)
    A, b = oracle_mod.posterior_system(prob)
    r = A @ mu.cpu().numpy().ravel() - b
    want_abs, bn = np.linalg.norm(r), np.linalg.norm(b)
    assert want_abs / bn > 1e-9      # far above the rounding of A mu - b
    assert abs(ab - want_abs) <= 1e-10 * want_abs + 1e-14 * bn
    assert abs(rel - want_abs / bn) <= 1e-10 * want_abs / bn + 1e-14
    G.gabp_destroy(ctx)


FP32_CASES = [
    (200, 150, 1, I.BC_NEUMANN, I.BC_NEUMANN, 1.0, 0.5, 0.2, 300),
    (193, 130, 2, I.BC_PERIODIC, I.BC_NEUMANN, 10.0, 0.5, 0.05, 1000),
    (256, 64, 2, I.BC_NEUMANN, I.BC_NEUMANN, 10.0, 0.5, 0.05, 1000),
]


@pytest.mark.parametrize("case", FP32_CASES, ids=lambda c: f"{c[0]}x{c[1]}a{c[2]}")
def test_fp32_matches_oracle_at_equal_t(G, oracle_mod, case):
    nx, ny, alpha, bcx, bcy, c, eta, kappa, t = case
    prob = I.small_lattice(nx, ny, alpha, bc_x=bcx, bc_y=bcy, kappa=kappa, c=c, tracks=6,
                           run=4, sigma=0.05, seed=nx + ny, dtype="f32")
    ctx = G.gabp_create_problem(prob)
    og = oracle_mod.OracleGaBP.from_problem(prob)
    G.gabp_iterate(ctx, t, eta)
    og.iterate(t, eta)
    errs = compare(prob, og, gpu_state(G, ctx), 1e-5)
    print("fp32 errors", case, errs)


def test_fp32_converged_alpha1_mean_equals_direct_solve(G, oracle_mod):
    prob = I.small_lattice(96, 80, 1, kappa=0.2, c=1.0, frac=0.05, sigma=0.1, seed=5, dtype="f32")
    ctx = G.gabp_create_problem(prob)
    st, it, rel = G.gabp_solve(ctx, 100000, 0.5, 1e-8, 10)
    assert st == G.GABP_OK, (st, it, rel)
    A, b = oracle_mod.posterior_system(prob)
    exact = oracle_mod.direct_solve(A, b)
    mu, _ = G.gabp_posterior(ctx, want_var=False)
    assert rel_l2(mu.cpu().numpy(), exact) <= 1e-5


# --------------------------------------------------------------------------
# divergence
# --------------------------------------------------------------------------

@pytest.mark.parametrize("eta", [0.5, 0.8])
def test_divergence_detected_at_the_oracles_iteration(G, oracle_mod, eta):
    prob = I.small_lattice(16, 16, 2, kappa=0.05, c=1.0, frac=0.05, sigma=0.05, seed=7, dtype="f64")
    og = oracle_mod.OracleGaBP.from_problem(prob)
    assert og.iterate(50, eta) == oracle_mod.STATUS_DIVERGED
    ctx = G.gabp_create_problem(prob)
    G.gabp_iterate(ctx, 50, eta)
    it, st = G.gabp_iteration_count(ctx)
    assert st == G.GABP_E_DIVERGED and it == og.diverged_at
    with pytest.raises(G.GabpError):
        G.gabp_iterate(ctx, 1, eta)
    # the state is that of the diverged iteration, compared where finite
    prec, info = G.gabp_get_messages(ctx)
    d, y, x, e = plane_slot_map(prob, og.g)
    pg = prec.cpu().numpy()[d, y, x]
    fin = np.isfinite(pg) & np.isfinite(og.lam[e])
    np.testing.assert_allclose(pg[fin], og.lam[e][fin], rtol=1e-9)


def test_table2_pattern_on_gpu(G):
    import json
    with open(os.path.join(os.path.dirname(__file__), "golden", "table2_divergence.json")) as f:
        gold = json.load(f)
    for eta_s, row in gold["diverged"].items():
        for c, want in zip(gold["c_values"], row):
            prob = I.small_lattice(32, 32, 2, kappa=0.074, c=float(c), frac=0.05, sigma=0.05,
                                   seed=7, dtype="f64")
            ctx = G.gabp_create_problem(prob)
            st, it, rel = G.gabp_solve(ctx, 3000, float(eta_s), 0.0, 20)
            got = st == G.GABP_E_DIVERGED
            assert got == want, (eta_s, c, st, it, rel)


# --------------------------------------------------------------------------
# state semantics: composition, checkpoint/resume, determinism, invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_iterations_compose_and_checkpoint_resume_bitwise(G, dtype):
    prob = I.small_lattice(150, 70, 2, bc_x=I.BC_PERIODIC, kappa=0.1, c=10.0, frac=0.1,
                           sigma=0.05, seed=3, dtype=dtype)
    a = G.gabp_create_problem(prob)
    G.gabp_iterate(a, 40, 0.5)
    ref = [t.cpu() for t in G.gabp_get_messages(a)]
    b = G.gabp_create_problem(prob)
    G.gabp_iterate(b, 15, 0.5)
    G.gabp_iterate(b, 5, 0.5)
    mid = G.gabp_get_messages(b)
    c = G.gabp_create_problem(prob)
    G.gabp_set_messages(c, *mid)
    G.gabp_iterate(c, 20, 0.5)
    G.gabp_iterate(b, 20, 0.5)
    for ctx in (b, c):
        got = [t.cpu() for t in G.gabp_get_messages(ctx)]
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])


def test_precision_messages_do_not_depend_on_data_and_information_is_linear(G):
    base = I.small_lattice(90, 60, 2, kappa=0.1, c=10.0, frac=0.1, sigma=0.05, seed=4, dtype="f64")
    outs = {}
    for k, s in (("1", 1.0), ("2", 2.0)):
        pr = I.Problem("lin", base.nx, base.ny, base.bc_x, base.bc_y, 2, base.kappa, base.tau,
                       base.c, base.sigma, base.cells, base.y * s, dtype="f64")
        ctx = G.gabp_create_problem(pr)
        G.gabp_iterate(ctx, 50, 0.5)
        outs[k] = [t.cpu() for t in G.gabp_get_messages(ctx)]
    assert torch.equal(outs["1"][0], outs["2"][0])
    assert torch.equal(outs["2"][1], 2 * outs["1"][1])


def test_message_change_statistic_matches_oracle(G, oracle_mod):
    prob = I.small_lattice(40, 30, 2, kappa=0.2, c=10.0, frac=0.1, sigma=0.05, seed=12, dtype="f64")
    ctx = G.gabp_create_problem(prob)
    G.gabp_iterate(ctx, 25, 0.5)
    r = G.gabp_message_change(ctx)
    og = oracle_mod.OracleGaBP.from_problem(prob)
    og.iterate(1, 0.5)
    m1 = (og.lam.copy(), og.th.copy())
    og.iterate(1, 0.5)
    m2 = (og.lam.copy(), og.th.copy())
    og.iterate(22, 0.5)
    prev = (og.lam.copy(), og.th.copy())
    og.iterate(1, 0.5)
    assert r == pytest.approx(og.early_stop_statistic(prev, m1, m2), rel=1e-10)


@pytest.mark.parametrize("dtype,alpha", [("f32", 2), ("f64", 1), ("f32", 1)])
def test_graph_chunks_equal_direct_launches(G, dtype, alpha):
    """gabp_solve replays recorded chunk graphs (eager checks, freeze probes
    and gain set-up between the replays); the result equals launching every
    kernel directly, bit for bit, before and after the precision messages
    froze (two-iteration launches inside the graphs)."""
    # the frozen-phase test's problem: its precision messages freeze bitwise
    # in every precision and order
    prob = I.small_lattice(190, 130, alpha, bc_x=I.BC_PERIODIC, kappa=0.1, tracks=5, run=4,
                           sigma=0.05, seed=77, dtype=dtype)
    a = G.gabp_create_problem(prob)
    b = G.gabp_create_problem(prob)
    G.gabp_set_graph(b, False)
    ra = G.gabp_solve(a, 600, 0.5, 0.0, 10)
    rb = G.gabp_solve(b, 600, 0.5, 0.0, 10)
    assert ra == rb and ra[1] == 600
    assert G.gabp_precision_frozen(a) == G.gabp_precision_frozen(b) > 0
    pa, ia = G.gabp_get_messages(a)
    pb, ib = G.gabp_get_messages(b)
    assert torch.equal(pa, pb) and torch.equal(ia, ib)
    # adaptive chunks (powers of two with graphs) against plain iterations
    c = G.gabp_create_problem(prob)
    st, it, rel = G.gabp_solve(c, 100000, 0.5, 1e-5 if dtype == "f32" else 1e-9, -10)
    assert st == G.GABP_OK
    d = G.gabp_create_problem(prob)
    G.gabp_iterate(d, it, 0.5)
    assert torch.equal(G.gabp_get_messages(c)[1], G.gabp_get_messages(d)[1])


def test_divergence_inside_a_replayed_chunk(G, oracle_mod):
    """A run that diverges inside a replayed chunk graph reports the oracle's
    iteration (numbered from the device counter) and keeps the messages of
    that iteration."""
    # c = 2 with learning rate 0.2 diverges at iteration 19 (oracle)
    prob = I.small_lattice(16, 16, 2, kappa=0.05, c=2.0, frac=0.05, sigma=0.05, seed=7, dtype="f64")
    og = oracle_mod.OracleGaBP.from_problem(prob)
    assert og.iterate(200, 0.2) == oracle_mod.STATUS_DIVERGED
    ctx = G.gabp_create_problem(prob)
    st, it, _ = G.gabp_solve(ctx, 200, 0.2, 0.0, 4)
    assert st == G.GABP_E_DIVERGED and it == og.diverged_at and it > 8
    prec, _ = G.gabp_get_messages(ctx)
    d, y, x, e = plane_slot_map(prob, og.g)
    pg = prec.cpu().numpy()[d, y, x]
    fin = np.isfinite(pg) & np.isfinite(og.lam[e])
    assert fin.sum() > 100
    np.testing.assert_allclose(pg[fin], og.lam[e][fin], rtol=1e-9)


def test_early_stop_rule_stops_where_the_oracle_does(G, oracle_mod):
    """The paper's early stop (mean |m^t - m^(t-1)| < tau mean |m^2 - m^1|),
    checked every iteration, ends at the first iteration where the oracle's
    statistic falls below tau; checked adaptively, it ends later but with
    the oracle's statistic at that iteration below tau."""
    prob = I.small_lattice(40, 30, 2, kappa=0.2, c=10.0, frac=0.1, sigma=0.05, seed=12, dtype="f64")
    tau = 1e-3
    og = oracle_mod.OracleGaBP.from_problem(prob)
    og.iterate(1, 0.5)
    m1 = (og.lam.copy(), og.th.copy())
    og.iterate(1, 0.5)
    m2 = (og.lam.copy(), og.th.copy())
    ratios = {}
    t = 2
    while t < 3000:
        prev = (og.lam.copy(), og.th.copy())
        og.iterate(1, 0.5)
        t += 1
        ratios[t] = og.early_stop_statistic(prev, m1, m2)
        if ratios[t] < tau:
            break
    t_stop = t
    assert ratios[t_stop] < tau and 50 < t_stop < 3000
    ctx = G.gabp_create_problem(prob)
    st, it, r = G.gabp_solve_early_stop(ctx, 5000, 0.5, tau, 1)
    assert st == G.GABP_OK and it == t_stop
    assert r == pytest.approx(ratios[t_stop], rel=1e-9)
    ctx2 = G.gabp_create_problem(prob)
    st, it2, r2 = G.gabp_solve_early_stop(ctx2, 5000, 0.5, tau, -5)
    assert st == G.GABP_OK and it2 >= t_stop and r2 < tau
    ctx3 = G.gabp_create_problem(prob)
    st, it3, _ = G.gabp_solve_early_stop(ctx3, 40, 0.5, tau, 1)
    assert st == G.GABP_E_NOT_CONVERGED and it3 == 40


def test_no_observations_gives_zero_mean(G):
    prob = I.Problem("empty", 40, 30, I.BC_NEUMANN, I.BC_NEUMANN, 2, 0.2, 1.0, 10.0, 0.1,
                     np.zeros(0, np.int64), np.zeros(0), dtype="f64")
    ctx = G.gabp_create_problem(prob)
    st, it, rel = G.gabp_solve(ctx, 100, 0.5, 1e-10, 10)
    assert st == G.GABP_OK and rel == 0.0
    mu, var = G.gabp_posterior(ctx)
    assert torch.count_nonzero(mu).item() == 0 and bool(torch.all(var > 0))


def test_duplicate_observations_add(G, oracle_mod):
    cells = np.array([5, 5, 17, 300, 5], dtype=np.int64)
    y = np.array([1.0, -0.5, 2.0, 0.3, 0.25])
    var = np.array([0.1, 0.2, 0.05, 0.3, 0.4])
    prob = I.Problem("dup", 25, 20, I.BC_NEUMANN, I.BC_NEUMANN, 1, 0.3, 1.0, 1.0, 0.1, cells, y,
                     var=var, dtype="f64")
    ctx = G.gabp_create_problem(prob)
    og = oracle_mod.OracleGaBP.from_problem(prob)
    G.gabp_iterate(ctx, 30, 0.5)
    og.iterate(30, 0.5)
    compare(prob, og, gpu_state(G, ctx), 1e-12)


def test_invalid_device_observations_rejected(G):
    grid = G._grid(16, 16)
    sten = G._stencil(1, 0.2, 1.0, 1.0)
    with pytest.raises(G.GabpError) as ei:
        G.gabp_create(grid, sten, torch.tensor([3, 256]), torch.tensor([1.0, 2.0]), 0.1)
    assert ei.value.status == G.GABP_E_INVALID
    with pytest.raises(G.GabpError) as ei:
        G.gabp_create(grid, sten, torch.tensor([3]), torch.tensor([float("nan")]), 0.1)
    assert ei.value.status == G.GABP_E_INVALID


def test_prior_mean_shifts_information(G, oracle_mod):
    prob = I.small_lattice(30, 20, 2, kappa=0.3, c=10.0, frac=0.2, sigma=0.1, seed=6, dtype="f64")
    fb = np.random.default_rng(0).normal(size=(prob.ny, prob.nx))
    ctx = G.gabp_create_problem(prob, prior_mean=torch.tensor(fb))
    og = oracle_mod.OracleGaBP.from_problem(prob, prior_mean=fb)
    G.gabp_iterate(ctx, 40, 0.5)
    og.iterate(40, 0.5)
    compare(prob, og, gpu_state(G, ctx), 1e-12)


# --------------------------------------------------------------------------
# full size, in the benchmark's launch configuration: sampled windows
# --------------------------------------------------------------------------

def _crop_problem(prob, x0, y0, w, h):
    """Sub-problem on columns x0..x0+w-1 (mod nx) and rows y0..y0+h-1 with the
    observations that fall inside.  Every crop edge is zero-flux: that is the
    real boundary of the global grid's y axis, and artificial edges lie
    outside the dependence cone of the compared window."""
    xs = (np.arange(x0, x0 + w) % prob.nx)
    ys = np.arange(y0, y0 + h)
    cx, cy = prob.cells % prob.nx, prob.cells // prob.nx
    colpos = np.full(prob.nx, -1)
    colpos[xs] = np.arange(w)
    inside = (colpos[cx] >= 0) & (cy >= y0) & (cy < y0 + h)
    cells = (cy[inside] - y0) * w + colpos[cx[inside]]
    assert prob.bc_y == I.BC_NEUMANN
    return I.Problem("crop", w, h, I.BC_NEUMANN, I.BC_NEUMANN,
                     prob.alpha, prob.kappa, prob.tau, prob.c, prob.sigma, cells, prob.y[inside],
                     dtype="f64")


def test_global8192_sampled_windows_match_oracle(G, oracle_mod):
    """8192x4096 FP32 run of 10 iterations; a message at iteration t depends
    only on data within 2t cells, so oracle runs on crops with a 2t + 4 margin
    reproduce the interior of each window (including the periodic seam and
    the zero-flux top and bottom rows, which the crops contain)."""
    prob = I.global8192()
    t = 10
    ctx = G.gabp_create_problem(prob)
    G.gabp_iterate(ctx, t, prob.damping)
    mean, _ = G.gabp_posterior(ctx, want_var=False)
    prec, info = G.gabp_get_messages(ctx)
    torch.cuda.synchronize()
    m = 2 * t + 4
    w = 48
    for (wx, wy) in ((4000, 2000), (8192 - 20, 1000), (100, 0), (6000, 4096 - w)):
        x0 = wx - m
        y0 = max(0, wy - m)
        y1 = min(prob.ny, wy + w + m)
        sub = _crop_problem(prob, x0, y0, w + 2 * m, y1 - y0)
        og = oracle_mod.OracleGaBP.from_problem(sub)
        og.iterate(t, prob.damping)
        mu_o, _ = og.posterior()
        mu_o = mu_o.reshape(sub.ny, sub.nx)[wy - y0: wy - y0 + w, m: m + w]
        cols = np.arange(wx, wx + w) % prob.nx
        mu_g = mean[wy: wy + w][:, cols].cpu().numpy()
        assert rel_l2(mu_g, mu_o) <= 1e-5, (wx, wy, rel_l2(mu_g, mu_o))
        lam_g = prec[:, wy: wy + w][:, :, cols].cpu().double().numpy()
        sd, sy, sx, e = plane_slot_map(sub, og.g)
        sel = (sy >= wy - y0) & (sy < wy - y0 + w) & (sx >= m) & (sx < m + w)
        assert rel_l2(lam_g[sd[sel], sy[sel] - (wy - y0), sx[sel] - m], og.lam[e[sel]]) <= 1e-5


@pytest.mark.parametrize("pair", [12, 16])
def test_global8192_two_iteration_kernel_is_bitwise_identical(G, pair):
    """The 8192 x 4096 workload in the configurations the benchmark times
    (12- and 16-row two-iteration tiles, ring and interior paths, once the
    precision messages froze): every message equals the single-iteration
    kernel's after the same iterations."""
    prob = I.global8192()
    a = G.gabp_create_problem(prob)
    b = G.gabp_create_problem(prob)
    G.gabp_set_tile(a, 1, pair)
    G.gabp_set_tile(b, 1, 0)
    fa, fb = _freeze(G, a), _freeze(G, b)
    assert fa == fb > 0
    w0 = G.gabp_launch_counts(a)["pair_tiles"]
    for n in (21, 2):
        G.gabp_iterate(a, n, prob.damping)
        G.gabp_iterate(b, n, prob.damping)
    assert G.gabp_launch_counts(a)["pair_tiles"] == w0 + 10
    assert G.gabp_iteration_count(a) == G.gabp_iteration_count(b)
    pa, ia = G.gabp_get_messages(a)
    pb, ib = G.gabp_get_messages(b)
    assert torch.equal(pa, pb)
    del pa, pb
    assert torch.equal(ia, ib)
    del ia, ib
    assert G.gabp_residual(a) == G.gabp_residual(b)
    G.gabp_destroy(a)
    G.gabp_destroy(b)


@pytest.mark.parametrize("dtype,alpha", [("f32", 2), ("f64", 1), ("f32", 1)])
def test_tile_shapes_are_bitwise_identical(G, dtype, alpha):
    """The autotuner runs real iterations with every tile shape; the result
    must equal the same number of iterations with the default shape."""
    prob = I.small_lattice(200, 75, alpha, bc_x=I.BC_PERIODIC, kappa=0.1, frac=0.1, sigma=0.05,
                           seed=31, dtype=dtype)
    a = G.gabp_create_problem(prob)
    G.gabp_iterate(a, 3, 0.5)
    chosen = G.gabp_autotune(a, 5, 0.5)
    assert chosen in (1, 2, 4, 8)
    assert G.gabp_iteration_count(a) == (3 + 1 + 8 * 5, G.GABP_OK)
    b = G.gabp_create_problem(prob)
    G.gabp_iterate(b, 3 + 1 + 8 * 5, 0.5)
    pa, ia = G.gabp_get_messages(a)
    pb, ib = G.gabp_get_messages(b)
    assert torch.equal(pa, pb) and torch.equal(ia, ib)


@pytest.mark.parametrize("dtype,alpha,n", [("f32", 2, 600), ("f64", 1, 400), ("f32", 1, 400)])
def test_frozen_precision_phase_is_bitwise_identical(G, dtype, alpha, n):
    """Residual checks detect when the precision messages stop changing and
    switch to the information-only kernel; the result must equal a run that
    never checks (full kernel throughout), bit for bit."""
    prob = I.small_lattice(190, 130, alpha, bc_x=I.BC_PERIODIC, kappa=0.1, tracks=5, run=4,
                           sigma=0.05, seed=77, dtype=dtype)
    a = G.gabp_create_problem(prob)
    for _ in range(n // 10):
        G.gabp_iterate(a, 10, 0.5)
        G.gabp_residual(a)
    frozen = G.gabp_precision_frozen(a)
    b = G.gabp_create_problem(prob)
    G.gabp_iterate(b, n, 0.5)
    pa, ia = G.gabp_get_messages(a)
    pb, ib = G.gabp_get_messages(b)
    print("frozen at", frozen)
    assert frozen > 0
    assert torch.equal(pa, pb) and torch.equal(ia, ib)


def _freeze(G, ctx):
    while G.gabp_precision_frozen(ctx) < 0:
        G.gabp_iterate(ctx, 10, 0.5)
        G.gabp_residual(ctx)
        assert G.gabp_iteration_count(ctx)[0] < 5000
    return G.gabp_precision_frozen(ctx)


@pytest.mark.parametrize("dtype,alpha,pair,nx,ny,bcx,bcy", [
    ("f32", 2, -4, 130, 23, I.BC_NEUMANN, I.BC_NEUMANN),
    ("f32", 2, -2, 70, 37, I.BC_PERIODIC, I.BC_NEUMANN),
    ("f32", 2, -8, 67, 40, I.BC_DIRICHLET, I.BC_PERIODIC),
    ("f32", 2, -4, 200, 17, I.BC_PERIODIC, I.BC_PERIODIC),
    ("f32", 2, -8, 150, 70, I.BC_NEUMANN, I.BC_DIRICHLET),
    ("f32", 2, -4, 257, 301, I.BC_PERIODIC, I.BC_NEUMANN),
    ("f32", 2, -2, 5, 70, I.BC_NEUMANN, I.BC_PERIODIC),
    ("f32", 2, -4, 9, 9, I.BC_PERIODIC, I.BC_PERIODIC),
    ("f32", 1, -4, 70, 40, I.BC_DIRICHLET, I.BC_PERIODIC),
    ("f32", 1, -8, 129, 45, I.BC_PERIODIC, I.BC_DIRICHLET),
    ("f32", 1, -2, 100, 50, I.BC_NEUMANN, I.BC_PERIODIC),
    ("f64", 2, -2, 140, 30, I.BC_PERIODIC, I.BC_NEUMANN),
    ("f64", 1, -2, 190, 130, I.BC_PERIODIC, I.BC_NEUMANN),
    ("f32", 2, 8, 130, 23, I.BC_NEUMANN, I.BC_NEUMANN),
    ("f32", 2, 4, 70, 37, I.BC_PERIODIC, I.BC_NEUMANN),
    ("f32", 2, 8, 67, 40, I.BC_DIRICHLET, I.BC_PERIODIC),
    ("f32", 2, 16, 200, 17, I.BC_PERIODIC, I.BC_PERIODIC),
    ("f32", 2, 16, 150, 70, I.BC_NEUMANN, I.BC_DIRICHLET),
    ("f32", 2, 32, 140, 75, I.BC_PERIODIC, I.BC_NEUMANN),
    ("f32", 2, 12, 150, 70, I.BC_NEUMANN, I.BC_DIRICHLET),
    ("f32", 2, 12, 132, 28, I.BC_NEUMANN, I.BC_PERIODIC),   # one interior tile
    # large lattices: most workgroups on the interior path, the ring a few
    # per cent of the nodes
    ("f32", 2, 16, 4096, 2048, I.BC_NEUMANN, I.BC_DIRICHLET),
    ("f32", 2, 12, 4100, 2060, I.BC_PERIODIC, I.BC_PERIODIC),
    ("f64", 2, 4, 4096, 2048, I.BC_NEUMANN, I.BC_NEUMANN),
    ("f32", 2, 12, 200, 41, I.BC_PERIODIC, I.BC_PERIODIC),
    ("f32", 2, 12, 300, 130, I.BC_NEUMANN, I.BC_NEUMANN),
    ("f32", 2, 12, 67, 23, I.BC_DIRICHLET, I.BC_PERIODIC),
    ("f32", 1, 12, 129, 45, I.BC_PERIODIC, I.BC_DIRICHLET),
    ("f32", 2, 8, 300, 130, I.BC_PERIODIC, I.BC_NEUMANN),
    ("f32", 1, 32, 70, 40, I.BC_DIRICHLET, I.BC_PERIODIC),
    ("f32", 2, 4, 5, 70, I.BC_NEUMANN, I.BC_PERIODIC),
    ("f32", 1, 8, 129, 45, I.BC_PERIODIC, I.BC_DIRICHLET),
    ("f32", 1, 16, 100, 50, I.BC_NEUMANN, I.BC_PERIODIC),
    ("f64", 2, 4, 140, 30, I.BC_PERIODIC, I.BC_NEUMANN),
    ("f64", 1, 4, 190, 130, I.BC_PERIODIC, I.BC_NEUMANN),
])
def test_two_iteration_kernel_is_bitwise_identical(G, dtype, alpha, pair, nx, ny, bcx, bcy):
    """Once the precision messages froze, two information-only iterations per
    launch (LDS halo, ragged and wrapped tiles) give bit for bit the messages,
    means and message-change statistic of one iteration per launch."""
    if (dtype, alpha) == ("f64", 1):
        # FP64 precision messages of the 5-point prior freeze bitwise only on
        # some problems; this is the frozen-phase test's, which does
        prob = I.small_lattice(nx, ny, alpha, bc_x=bcx, bc_y=bcy, kappa=0.1, tracks=5, run=4,
                               sigma=0.05, seed=77, dtype=dtype)
    else:
        prob = I.small_lattice(nx, ny, alpha, bc_x=bcx, bc_y=bcy, kappa=0.12, frac=0.08,
                               sigma=0.05, seed=nx + ny, dtype=dtype)
    a = G.gabp_create_problem(prob)
    b = G.gabp_create_problem(prob)
    G.gabp_set_tile(a, 4, pair)
    G.gabp_set_tile(b, 4, 0)
    assert G.gabp_get_tile(a) == (4, pair)
    if nx * ny > 30000:
        # a few FP32 precision messages of this lattice keep flipping their
        # last bit; both contexts freeze them at the same iteration
        G.gabp_set_freeze_tolerance(a, 64, 1e-6)
        G.gabp_set_freeze_tolerance(b, 64, 1e-6)
    fa, fb = _freeze(G, a), _freeze(G, b)
    assert fa == fb > 0
    before = G.gabp_launch_counts(a)
    for n in (41, 3, 2, 1, 16):
        G.gabp_iterate(a, n, 0.5)
        G.gabp_iterate(b, n, 0.5)
        pa, ia = G.gabp_get_messages(a)
        pb, ib = G.gabp_get_messages(b)
        assert torch.equal(pa, pb) and torch.equal(ia, ib), n
        assert G.gabp_message_change(a) == G.gabp_message_change(b)
    ma, _ = G.gabp_posterior(a, want_var=False)
    mb, _ = G.gabp_posterior(b, want_var=False)
    assert torch.equal(ma, mb)
    assert G.gabp_iteration_count(a) == G.gabp_iteration_count(b)
    # the kernel under test did run: 41, 3, 2, 1 and 16 iterations are 20 + 1
    # + 0 + 0 + 7 two-iteration launches and 7 single ones
    after = G.gabp_launch_counts(a)
    kind, other = ("pair_tiles", "pair_walk") if pair > 0 else ("pair_walk", "pair_tiles")
    assert after[kind] - before[kind] == 28 and after[other] == before[other]
    assert after["theta"] - before["theta"] == 7 and after["full"] == before["full"]


def test_autotune_after_freezing_times_the_two_iteration_kernel(G):
    prob = I.small_lattice(150, 60, 2, kappa=0.12, frac=0.08, sigma=0.05, seed=3, dtype="f32")
    a = G.gabp_create_problem(prob)
    _freeze(G, a)
    t0 = G.gabp_iteration_count(a)[0]
    G.gabp_autotune(a, 5, 0.5)
    # 5 tile heights, twice each, after the single shapes
    assert G.gabp_iteration_count(a)[0] == t0 + 1 + 8 * 5 + 10 * 5
    rpt, pair = G.gabp_get_tile(a)
    assert rpt in (1, 2, 4, 8) and pair in (0, 4, 8, 12, 16, 32)
    b = G.gabp_create_problem(prob)
    G.gabp_set_tile(b, 4, 0)
    _freeze(G, b)
    G.gabp_iterate(b, 1 + 8 * 5 + 10 * 5, 0.5)
    assert torch.equal(G.gabp_get_messages(a)[1], G.gabp_get_messages(b)[1])
    with pytest.raises(G.GabpError):
        G.gabp_set_tile(a, 3, 0)
    with pytest.raises(G.GabpError):
        G.gabp_set_tile(G.gabp_create_problem(I.small_lattice(20, 20, 2, dtype="f64")), 4, 8)
    with pytest.raises(G.GabpError):
        G.gabp_set_tile(G.gabp_create_problem(I.small_lattice(20, 20, 2, dtype="f64")), 4, -4)
    with pytest.raises(G.GabpError):
        G.gabp_set_tile(a, 4, -3)


# --------------------------------------------------------------------------
# batched instances
# --------------------------------------------------------------------------

def _mixed_problems(dtype, n=9):
    out = []
    specs = [(70, 66, 1, I.BC_NEUMANN, I.BC_NEUMANN), (130, 40, 2, I.BC_PERIODIC, I.BC_NEUMANN),
             (33, 90, 2, I.BC_NEUMANN, I.BC_DIRICHLET), (64, 64, 1, I.BC_PERIODIC, I.BC_PERIODIC),
             (200, 17, 2, I.BC_NEUMANN, I.BC_NEUMANN), (5, 300, 2, I.BC_NEUMANN, I.BC_NEUMANN),
             (97, 101, 2, I.BC_DIRICHLET, I.BC_NEUMANN), (1, 64, 1, I.BC_NEUMANN, I.BC_NEUMANN),
             (150, 120, 2, I.BC_NEUMANN, I.BC_PERIODIC)]
    for k, (nx, ny, a, bx, by) in enumerate(specs[:n]):
        out.append(I.small_lattice(nx, ny, a, bc_x=bx, bc_y=by, kappa=0.1 + 0.03 * k,
                                   frac=0.04 + 0.02 * k, sigma=0.05 + 0.01 * k, seed=500 + k,
                                   dtype=dtype))
    return out


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_iterations_bitwise_equal_single_contexts(G, dtype):
    probs = _mixed_problems(dtype)
    b = G.gabp_batch_create(probs)
    G.gabp_batch_iterate(b, 37, 0.5)
    for i, p in enumerate(probs):
        ctx = G.gabp_create_problem(p)
        G.gabp_iterate(ctx, 37, 0.5)
        pa, ia = G.gabp_batch_get_messages(b, i)
        pb, ib = G.gabp_get_messages(ctx)
        assert torch.equal(pa, pb) and torch.equal(ia, ib), i


def test_batch_solve_matches_single_solves(G, oracle_mod):
    """Per-instance convergence, retirement and freezing through the captured
    chunk graph: iteration counts, final messages and means equal the
    single-context solves bit for bit; every mean is within 1 % of the
    direct solve of the oracle's posterior system (the FP64 oracle iterated
    to the same 1e-6 residual is 2e-4 to 2.4e-3 from it on these problems:
    the residual understates a slowly converging error); a diverging
    instance (13-point prior with c = 1) is reported with the oracle's
    iteration."""
    probs = _mixed_problems("f32", 7)
    bad = I.small_lattice(16, 16, 2, kappa=0.05, c=1.0, frac=0.05, sigma=0.05, seed=7, dtype="f32")
    probs.append(bad)
    b = G.gabp_batch_create(probs)
    st, its, rels, sts = G.gabp_batch_solve(b, 60000, 0.5, 1e-6, 10)
    assert sts[-1] == G.GABP_E_DIVERGED
    og = oracle_mod.OracleGaBP.from_problem(bad)
    og.iterate(50, 0.5)
    assert its[-1] == og.diverged_at
    for i, p in enumerate(probs[:-1]):
        assert sts[i] == G.GABP_OK, (i, sts[i], rels[i])
        ctx = G.gabp_create_problem(p)
        s1, it1, rel1 = G.gabp_solve(ctx, 60000, 0.5, 1e-6, 10)
        assert s1 == G.GABP_OK and it1 == its[i], (i, it1, its[i])
        assert rel1 == pytest.approx(rels[i], rel=1e-9)
        pa, ia = G.gabp_batch_get_messages(b, i)
        pb, ib = G.gabp_get_messages(ctx)
        assert torch.equal(pa, pb) and torch.equal(ia, ib), i
        assert G.gabp_batch_info(b, i)[1] == G.gabp_precision_frozen(ctx)
        mu, _ = G.gabp_batch_posterior(b, i, want_var=False)
        mref, _ = G.gabp_posterior(ctx, want_var=False)
        assert torch.equal(mu, mref)
        A, rhs = oracle_mod.posterior_system(p)
        exact = oracle_mod.direct_solve(A, rhs)
        assert rel_l2(mu.cpu().numpy().ravel(), exact) <= 1e-2, i


def test_freeze_tolerance_freezes_precisions_that_keep_flipping(G, oracle_mod):
    """Instance 168 of the uneven batch (277^2, 13-point prior): a few FP32
    precision messages keep changing in their last bit, so the bitwise test
    never freezes them.  With a tolerance of 64 messages changed by at most
    1e-6 (relative) they freeze, the solve still reaches the residual
    tolerance, and the mean is as close to the direct solve as the unfrozen
    run's."""
    p = I.batch256_instance(168)
    strict = G.gabp_create_problem(p)
    st, it, rel = G.gabp_solve(strict, 30000, 0.5, 1e-6, 10)
    assert st == G.GABP_OK and G.gabp_precision_frozen(strict) == -1, (st, it)
    relaxed = G.gabp_create_problem(p)
    with pytest.raises(G.GabpError):
        G.gabp_set_freeze_tolerance(relaxed, -1, 0.0)
    with pytest.raises(G.GabpError):
        G.gabp_set_freeze_tolerance(relaxed, 8, float("nan"))
    G.gabp_set_freeze_tolerance(relaxed, 64, 1e-6)
    st2, it2, rel2 = G.gabp_solve(relaxed, 30000, 0.5, 1e-6, 10)
    fz = G.gabp_precision_frozen(relaxed)
    assert st2 == G.GABP_OK and rel2 <= 1e-6
    assert 0 < fz < it2, (fz, it2)
    A, b = oracle_mod.posterior_system(p)
    exact = oracle_mod.direct_solve(A, b)
    e_s = rel_l2(G.gabp_posterior(strict, want_var=False)[0].cpu().numpy().ravel(), exact)
    e_r = rel_l2(G.gabp_posterior(relaxed, want_var=False)[0].cpu().numpy().ravel(), exact)
    assert e_r <= 2 * e_s + 1e-7, (e_r, e_s)
    G.gabp_destroy(strict)
    G.gabp_destroy(relaxed)


def test_batch_freeze_tolerance_matches_single_contexts(G):
    """The batch applies the same tolerance at the same checks as lone
    contexts: iteration counts, freezing iterations and final messages equal
    bit for bit, and the instance whose precisions keep flipping freezes."""
    probs = _mixed_problems("f32", 5) + [I.batch256_instance(168)]
    b = G.gabp_batch_create(probs)
    G.gabp_batch_set_freeze_tolerance(b, 64, 1e-6)
    st, its, rels, sts = G.gabp_batch_solve(b, 30000, 0.5, 1e-6, 10)
    for i, p in enumerate(probs):
        ctx = G.gabp_create_problem(p)
        G.gabp_set_freeze_tolerance(ctx, 64, 1e-6)
        s1, it1, _ = G.gabp_solve(ctx, 30000, 0.5, 1e-6, 10)
        assert sts[i] == G.GABP_OK and s1 == G.GABP_OK and it1 == its[i], (i, it1, its[i])
        assert G.gabp_batch_info(b, i)[1] == G.gabp_precision_frozen(ctx), i
        pa, ia = G.gabp_batch_get_messages(b, i)
        pb, ib = G.gabp_get_messages(ctx)
        assert torch.equal(pa, pb) and torch.equal(ia, ib), i
        G.gabp_destroy(ctx)
    assert G.gabp_batch_info(b, len(probs) - 1)[1] > 0
    G.gabp_batch_destroy(b)


def test_batch_adaptive_chunks_converge_and_stay_bitwise(G):
    """check_every < 0 grows the chunks once every running instance froze;
    every instance still reaches the tolerance, and its messages equal a lone
    context's after the same number of iterations, bit for bit."""
    probs = _mixed_problems("f32", 6)
    b = G.gabp_batch_create(probs)
    st, its, rels, sts = G.gabp_batch_solve(b, 60000, 0.5, 1e-6, -10)
    assert st == G.GABP_OK
    fixed = G.gabp_batch_create(probs)
    _, its_fixed, _, _ = G.gabp_batch_solve(fixed, 60000, 0.5, 1e-6, 10)
    for i, p in enumerate(probs):
        assert sts[i] == G.GABP_OK and rels[i] <= 1e-6, (i, sts[i], rels[i])
        assert its[i] >= its_fixed[i]
        ctx = G.gabp_create_problem(p)
        G.gabp_iterate(ctx, its[i], 0.5)
        pa, ia = G.gabp_batch_get_messages(b, i)
        pb, ib = G.gabp_get_messages(ctx)
        assert torch.equal(pa, pb) and torch.equal(ia, ib), i
    with pytest.raises(G.GabpError):
        G.gabp_batch_solve(b, 10, 0.5, 1e-6, 0)


def test_batch256_full_size_sampled_instances_bitwise(G):
    """The 256-instance workload in the benchmark's configuration (adaptive
    chunks, FP32, to 1e-6): every instance converges, and sampled instances
    (the smallest, a median one, the slowest) equal lone contexts run for the
    same number of iterations, bit for bit."""
    probs = I.batch256()
    b = G.gabp_batch_create(probs)
    st, its, rels, sts = G.gabp_batch_solve(b, 300000, 0.5, 1e-6, -10)
    assert st == G.GABP_OK and np.all(sts == G.GABP_OK) and np.all(rels <= 1e-6)
    sizes = np.array([p.n for p in probs])
    picks = {int(np.argmin(sizes)), int(np.argsort(its)[len(its) // 2]), int(np.argmax(its))}
    for i in sorted(picks):
        ctx = G.gabp_create_problem(probs[i])
        G.gabp_iterate(ctx, int(its[i]), 0.5)
        pa, ia = G.gabp_batch_get_messages(b, i)
        pb, ib = G.gabp_get_messages(ctx)
        assert torch.equal(pa, pb) and torch.equal(ia, ib), (i, its[i])
        G.gabp_destroy(ctx)
    G.gabp_batch_destroy(b)


def test_batch_autotune_keeps_results(G):
    probs = _mixed_problems("f32", 5)
    a = G.gabp_batch_create(probs)
    ch = G.gabp_batch_autotune(a, 2, 0.5)
    assert ch in (1, 2, 4, 8)
    b = G.gabp_batch_create(probs)
    G.gabp_batch_iterate(b, 1 + 8 * 2, 0.5)
    for i in range(len(probs)):
        pa, ia = G.gabp_batch_get_messages(a, i)
        pb, ib = G.gabp_batch_get_messages(b, i)
        assert torch.equal(pa, pb) and torch.equal(ia, ib)
