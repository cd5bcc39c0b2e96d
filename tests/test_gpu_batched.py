"""Batched fits of many uneven GLAMs (three batched launches per proximal step)
against the oracle, problem by problem."""
import numpy as np
import pytest

import oracle.glam_oracle as O
from paper_1510_03298_amd import inputs
from tests.gpu_util import need_gpu, rel_inf

pytestmark = pytest.mark.gpu


def _upload(glam, d):
    return {"X": [glam.to_device_colmajor(X, 0) for X in d.X], "Y": glam.to_device_colmajor(d.Y, 0),
            "n": d.n, "p": d.p, "family": d.family}


@pytest.mark.parametrize("dt", [1, 0])
def test_batched_mixed_families_match_oracle(dt):
    torch, glam = need_gpu()
    print(f"batched dt={dt}", flush=True)
    probs = inputs.config_c4(nprob=6, lo=16, hi=40, seed_offset=40)
    res = glam.fit_batched([_upload(glam, d) for d in probs], lambda_ratio=0.1, dtype=dt, kkt_tol=1e-6)
    assert res.code == 0 and np.all(res.status == 0)
    for i, d in enumerate(probs):
        fam = d.family
        lm = O.lambda_max(fam, d.X, d.Y)
        assert abs(res.lambda_max[i] - lm) <= 1e-12 * lm
        lam = 0.1 * lm
        th = glam.from_colmajor(res.theta[i], d.p)
        g = O.smooth_gradient(fam, d.X, th, d.Y)
        assert O.kkt_residual(th, g, lam, lm) <= 1e-6
        ref, info = O.gdpg(fam, d.X, d.Y, lam, lm, tol=1e-10, max_outer=200)   # the oracle from zero
        assert info.converged
        assert rel_inf(th, ref) <= 1e-3


def test_batched_matches_single_problem_fits():
    """The same PMLE as glam_fit_path on each problem alone."""
    torch, glam = need_gpu()
    probs = inputs.config_c4(nprob=4, lo=16, hi=32, seed_offset=41)
    ups = [_upload(glam, d) for d in probs]
    res = glam.fit_batched(ups, lambda_ratio=0.2, dtype=1, kkt_tol=1e-7)
    for i, d in enumerate(probs):
        r1 = glam.fit_path(ups[i]["X"], ups[i]["Y"], d.n, d.p, d.family, lambdas=[res.lambdas[i]], dtype=1,
                           kkt_tol=1e-7)
        a = glam.from_colmajor(res.theta[i], d.p)
        b = glam.from_colmajor(r1.theta[0], d.p)
        assert rel_inf(a, b) <= 1e-4


def test_batched_rejects_bad_problem():
    torch, glam = need_gpu()
    probs = inputs.config_c4(nprob=2, lo=16, hi=20, seed_offset=42)
    ups = [_upload(glam, d) for d in probs]
    ups[1]["family"] = 7
    with pytest.raises(glam.GlamError):
        glam.fit_batched(ups, lambda_ratio=0.1, dtype=1)


def test_batched_full_c4_sampled():
    """All 256 uneven problems (n_ij in 16..96) in one batch, FP32 inner chain;
    the KKT residual of a sample of problems recomputed by the oracle."""
    torch, glam = need_gpu()
    probs = inputs.config_c4()
    ups = [_upload(glam, d) for d in probs]
    res = glam.fit_batched(ups, lambda_ratio=0.1, dtype=1, kkt_tol=1e-6)
    assert res.code == 0 and np.all(res.status == 0)
    assert np.all(res.kkt <= 1e-6)
    rng = np.random.default_rng(7)
    for i in sorted(rng.choice(len(probs), size=6, replace=False)):
        d = probs[i]
        lm = O.lambda_max(d.family, d.X, d.Y)
        th = glam.from_colmajor(res.theta[i], d.p)
        g = O.smooth_gradient(d.family, d.X, th, d.Y)
        assert O.kkt_residual(th, g, 0.1 * lm, lm) <= 1e-6, i


def test_batched_elastic_net():
    """Sec. 6.3 elastic net in the batched solver: the oracle's elastic-net KKT
    evaluator on every problem."""
    torch, glam = need_gpu()
    probs = inputs.config_c4(nprob=5, lo=16, hi=40, seed_offset=43)
    res = glam.fit_batched([_upload(glam, d) for d in probs], lambda_ratio=0.1, dtype=2, kkt_tol=1e-6, alpha=1.0)
    assert res.code == 0 and np.all(res.status == 0)
    for i, d in enumerate(probs):
        lm = O.lambda_max(d.family, d.X, d.Y)
        th = glam.from_colmajor(res.theta[i], d.p)
        g = O.smooth_gradient(d.family, d.X, th, d.Y)
        assert O.kkt_residual(th, g, 0.1 * lm, lm, alpha=1.0) <= 1e-6
        F = O.objective(d.family, d.X, th, d.Y, 0.1 * lm, alpha=1.0)
        assert abs(res.objective[i] - F) <= 1e-9 * abs(F)


def test_batched_four_families():
    """One batch mixing all four families (Gaussian, Poisson, Binomial, Gamma)."""
    torch, glam = need_gpu()
    fams = ["gaussian", "poisson", "binomial", "gamma"] * 2
    probs = [inputs.random_problem((17 + 3 * i, 20 + i, 19 + 2 * i), (5, 6, 5), family=f, seed=50 + i,
                                   basis="gauss", scale=0.3) for i, f in enumerate(fams)]
    res = glam.fit_batched([_upload(glam, d) for d in probs], lambda_ratio=0.1, dtype=1, kkt_tol=1e-6)
    assert res.code == 0 and np.all(res.status == 0)
    for i, d in enumerate(probs):
        lm = O.lambda_max(d.family, d.X, d.Y)
        th = glam.from_colmajor(res.theta[i], d.p)
        g = O.smooth_gradient(d.family, d.X, th, d.Y)
        assert O.kkt_residual(th, g, 0.1 * lm, lm) <= 1e-6, (i, d.family)


@pytest.mark.parametrize("dt", [1, 0])
@pytest.mark.parametrize("fam", ["gaussian", "poisson"])
def test_batched_mode_order_chosen_by_the_library(fam, dt):
    """A batch holding Section 6.5's design in the paper's own mode order (60r, 20r, 10r), r = 2,
    whose p_1 = 60 does not fit the slab kernels: the batched solver reorders that problem itself.
    Bit for bit the estimates of the same batch with the problem given in an order that fits, and
    the oracle's KKT on the caller's order."""
    torch, glam = need_gpu()
    d = inputs.config_sim(r=2, family=fam, seed=9)            # listed as (20r, 10r, 60r)
    Xs = [d.X[2], d.X[0], d.X[1]]                             # the paper's order
    Y = np.asfortranarray(d.Y.transpose(2, 0, 1))
    n = tuple(X.shape[0] for X in Xs)
    p = tuple(X.shape[1] for X in Xs)
    other = inputs.config_c4(nprob=1, lo=16, hi=24, seed_offset=43)[0]
    print(f"batched mode order {fam} dt={dt} n={n} p={p}", flush=True)
    up = {"X": [glam.to_device_colmajor(X, 0) for X in Xs], "Y": glam.to_device_colmajor(Y, 0),
          "n": n, "p": p, "family": fam}
    up_fit = {"X": [glam.to_device_colmajor(X, 0) for X in d.X], "Y": glam.to_device_colmajor(d.Y, 0),
              "n": d.n, "p": d.p, "family": fam}
    r1 = glam.fit_batched([up, _upload(glam, other)], lambda_ratio=0.1, dtype=dt, kkt_tol=1e-7)
    r2 = glam.fit_batched([up_fit, _upload(glam, other)], lambda_ratio=0.1, dtype=dt, kkt_tol=1e-7)
    assert r1.code == r2.code == 0
    assert np.array_equal(r1.iters_outer, r2.iters_outer)
    a = glam.from_colmajor(r1.theta[0], p)
    b = glam.from_colmajor(r2.theta[0], d.p)
    assert np.array_equal(a, np.asfortranarray(b.transpose(2, 0, 1)))
    assert np.array_equal(glam.from_colmajor(r1.theta[1], other.p), glam.from_colmajor(r2.theta[1], other.p))
    lm = O.lambda_max(fam, Xs, Y)
    assert abs(r1.lambda_max[0] - lm) <= 1e-12 * lm
    g = O.smooth_gradient(fam, Xs, a, Y)
    assert O.kkt_residual(a, g, 0.1 * lm, lm) <= 1e-7


def test_batched_f32_lds_slab_path():
    """A batch with one problem beyond the register kernel (n_1 = 150 > 128) runs every slab phase
    on the workgroup-per-slab LDS kernel in FP32: each problem's KKT by the oracle."""
    torch, glam = need_gpu()
    probs = inputs.config_c4(nprob=2, lo=16, hi=30, seed_offset=44)
    big = inputs.random_problem((150, 20, 24), (12, 8, 6), family="poisson", seed=45, scale=0.3)
    ups = [_upload(glam, d) for d in probs] + [{"X": [glam.to_device_colmajor(X, 0) for X in big.X],
                                                "Y": glam.to_device_colmajor(big.Y, 0), "n": big.n, "p": big.p,
                                                "family": "poisson"}]
    print("batched f32 lds path", flush=True)
    res = glam.fit_batched(ups, lambda_ratio=0.1, dtype=1, kkt_tol=1e-6)
    assert res.code == 0 and np.all(res.status == 0)
    for i, (X, Y, p, fam) in enumerate([(d.X, d.Y, d.p, d.family) for d in probs] + [(big.X, big.Y, big.p, "poisson")]):
        lm = O.lambda_max(fam, X, Y)
        th = glam.from_colmajor(res.theta[i], p)
        assert O.kkt_residual(th, O.smooth_gradient(fam, X, th, Y), 0.1 * lm, lm) <= 1e-6, i


def test_batched_reports_the_invalid_problem():
    """Input checks run per problem on the device and are read by several host threads: a
    negative count in problem 3 (Poisson) is reported with that problem's index."""
    torch, glam = need_gpu()
    probs = inputs.config_c4(nprob=6, lo=16, hi=24, seed_offset=46)
    ups = [_upload(glam, d) for d in probs]
    assert probs[3].family == "poisson"
    ups[3]["Y"] = ups[3]["Y"].clone()
    ups[3]["Y"][5] = -1.0
    with pytest.raises(glam.GlamError) as e:
        glam.fit_batched(ups, lambda_ratio=0.1, dtype=1)
    assert "problem 3" in str(e.value) and "Poisson Y must be >= 0" in str(e.value)


@pytest.mark.parametrize("dt", [1, 2])
def test_batched_tuned_graph_matches_fixed_eager(dt, tmp_path, monkeypatch):
    """The tuner's slab-phase variants (run length, kernel width) and the graph replays compute the
    same values: tuned + graph and fixed + stream launches give bit-identical estimates.  The tuned
    choices are written to GLAM_TUNE_FILE and read back by a second tuned call (no new timing)."""
    torch, glam = need_gpu()
    tune = tmp_path / "tune.txt"
    monkeypatch.setenv("GLAM_TUNE_FILE", str(tune))
    probs = inputs.config_c4(nprob=24, lo=16, hi=96, seed_offset=43)
    ups = [_upload(glam, d) for d in probs]
    print(f"batched tuned vs fixed dt={dt}", flush=True)
    r1 = glam.fit_batched(ups, lambda_ratio=0.1, dtype=dt, kkt_tol=1e-6, tuning="auto", graph=True)
    r2 = glam.fit_batched(ups, lambda_ratio=0.1, dtype=dt, kkt_tol=1e-6, tuning="fixed", graph=False)
    assert r1.code == r2.code == 0
    assert r1.graph_replays > 0 and r2.graph_replays == 0
    for a, b in zip(r1.theta, r2.theta):
        assert torch.equal(a, b)
    assert np.array_equal(r1.iters_outer, r2.iters_outer)
    for i, d in enumerate(probs):
        lm = O.lambda_max(d.family, d.X, d.Y)
        th = glam.from_colmajor(r1.theta[i], d.p)
        assert O.kkt_residual(th, O.smooth_gradient(d.family, d.X, th, d.Y), 0.1 * lm, lm) <= 1e-6
    r3 = glam.fit_batched(ups, lambda_ratio=0.1, dtype=dt, kkt_tol=1e-6, tuning="auto", graph=True)
    assert r3.tune_seconds == 0.0   # every class signature already tuned in this process
    for a, b in zip(r1.theta, r3.theta):
        assert torch.equal(a, b)
