"""Captured passes of the single-image solve (a full extrapolation cycle, or one FP call with its
relative-change pass, recorded into a HIP graph on first use and replayed): replays give the
same iterates as the first, captured run; every setting a pass records invalidates it (the
operator, sigma, lambda, m, the SD step, the denoiser precision, CG iterations); a pass never
refers to the caller's observation buffer; image sizes share a handle."""
import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def say(*a):
    print(*a, flush=True)


def obs(torch, prob):
    import oracle
    y = np.asarray(oracle.OracleProblem(prob).y, dtype=np.float32)
    return torch.tensor(y, device="cuda")


def restorer(prob, **kw):
    from paper_1805_02158_amd import Restorer
    return Restorer(0).configure(prob, **kw)


def run(r, y, prob):
    x, st = r.solve(y, *prob.hr_shape)
    return x.cpu().numpy(), st


@pytest.mark.parametrize("method,L,m,calls", [("rre", 5, 0, 15), ("mpe", 4, 1, 15),
                                              ("none", 5, 0, 6)])
def test_replay_matches_capture_and_a_fresh_handle(torch, method, L, m, calls):
    prob = W.problem("deblur64")
    y = obs(torch, prob)
    r = restorer(prob, method=method, L=L, m=m, tol=0.0, max_fp_calls=calls)
    x1, s1 = run(r, y, prob)
    x2, s2 = run(r, y, prob)
    x3, s3 = run(restorer(prob, method=method, L=L, m=m, tol=0.0, max_fp_calls=calls), y, prob)
    say(f"  {method}: calls {s1['fp_calls']}, cycles {s1['cycles']}")
    assert s1 == {**s2, "ms": s1["ms"]} and s1["fp_calls"] == calls
    assert np.array_equal(x1, x2) and np.array_equal(x1, x3)


def test_new_observation_buffer_each_solve(torch):
    prob = W.problem("deblur64")
    y = obs(torch, prob)
    r = restorer(prob, method="rre", L=5, tol=0.0, max_fp_calls=10)
    ref, _ = run(r, y, prob)
    for scale in (1.0, 0.5):
        y2 = (y * scale).clone()  # a new allocation with new contents
        x, _ = run(r, y2, prob)
        fresh, _ = run(restorer(prob, method="rre", L=5, tol=0.0, max_fp_calls=10), y2, prob)
        assert np.array_equal(x, fresh)
    del y2
    x, _ = run(r, y, prob)
    assert np.array_equal(x, ref)


def _changes():
    return [("lambda", lambda r: r.set_lambda(0.03)),
            ("sigma", lambda r: r.set_noise(2.0)),
            ("operator", lambda r: r.set_operator(W.psf_uniform(5), 1)),
            ("m", lambda r: r.set_extrapolation("rre", 5, 1)),
            ("cg", lambda r: r.set_solver(8, 12, 0.0, 0)),
            ("bf16", lambda r: r.set_denoiser(W.make_denoiser(), "bf16")),
            ("sd step", lambda r: r.set_base("sd", 0.05))]


@pytest.mark.parametrize("name", [c[0] for c in _changes()])
def test_settings_invalidate_the_captured_pass(torch, name):
    change = dict(_changes())[name]
    prob = W.problem("deblur64")
    y = obs(torch, prob)
    r = restorer(prob, method="rre", L=5, tol=0.0, max_fp_calls=12)
    if name == "sd step":
        r.set_base("sd", 0.02)
    run(r, y, prob)
    change(r)
    x, _ = run(r, y, prob)
    f = restorer(prob, method="rre", L=5, tol=0.0, max_fp_calls=12)
    if name == "sd step":
        f.set_base("sd", 0.02)
    change(f)
    xf, _ = run(f, y, prob)
    assert np.array_equal(x, xf)


def test_sizes_share_a_handle(torch):
    from paper_1805_02158_amd import Restorer
    probs = [W.problem("deblur64"), W.problem("tiny"), W.problem("deblur64")]
    r = Restorer(0)
    outs = []
    for p in probs:
        r.configure(p, method="rre", L=5, tol=0.0, max_fp_calls=10)
        outs.append(run(r, obs(torch, p), p)[0])
    assert np.array_equal(outs[0], outs[2])
    fresh = run(restorer(probs[1], method="rre", L=5, tol=0.0, max_fp_calls=10),
                obs(torch, probs[1]), probs[1])[0]
    assert np.array_equal(outs[1], fresh)
