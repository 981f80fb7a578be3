"""The BF16 form's switch to FP32 banks (redve_set_precision_switch) through the C ABI: once an
image's relative change falls below the switch, its remaining FP calls take the FP32 banks and
the FP32 window. Checked against the FP64 oracle's fixed point at the FP32 bar, against the
solve without the switch (fewer or equal FP calls to the same tolerance), and in the batched
engine (per image equal to the single-image path, and bitwise the same alone and in a mix)."""
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


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.lib()
    return oracle


def say(*a):
    print(*a, flush=True)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def host(t):
    return t.detach().cpu().double().numpy()


@pytest.mark.parametrize("name,L", [("deblur256", 5), ("deblur64", 5), ("sr512", 8)])
def test_switch_converges_to_the_fixed_point(torch, orc, name, L):
    from paper_1805_02158_amd import Restorer
    prob = W.problem(name)
    y32 = f32(orc.OracleProblem(prob).y)
    ref = orc.solve(orc.OracleProblem(prob, y=y32), "rre", L=L, m=0, tol=1e-10, max_calls=300)
    out = {}
    for sw in (0.0, 1e-4):
        r = Restorer(0).configure(prob, precision="bf16", method="rre", L=L, m=0, tol=1e-5,
                                  max_fp_calls=400)
        r.set_precision_switch(sw)
        x, st = r.solve(dev(torch, y32), *prob.hr_shape)
        e = rel(host(x), ref.x)
        dp = orc.psnr(host(x), prob.x_true) - orc.psnr(ref.x, prob.x_true)
        say(f"  {name} switch {sw:g}: {st['fp_calls']} FP calls, rel L2 vs the fixed point "
            f"{e:.2e}, dPSNR {dp:+.4f} dB")
        assert st["status"] == 0 and abs(dp) <= 0.05
        out[sw] = (st["fp_calls"], e)
    # with the switch the last cycles run on FP32 banks: the FP32 bar
    assert out[1e-4][1] <= 1e-4
    assert out[1e-4][0] <= out[0.0][0]


def test_switch_in_the_batch(torch, orc):
    """Batched BF16 solves with the switch: each image equals its single-image solve with the
    switch, and is bitwise the same alone and in the mix (its switch depends on its own
    relative change only)."""
    from paper_1805_02158_amd import Restorer
    probs = [W.problem("deblur64"), W.problem("tiny"), W.problem("deblur256")]
    ys = [f32(orc.OracleProblem(p).y) for p in probs]
    rb = Restorer(0)
    rb.set_denoiser(W.make_denoiser(), "bf16").set_extrapolation("rre", 5, 0)
    rb.set_solver(15, 200, 1e-5, 0).set_precision_switch(1e-4)

    def items(idx):
        return [dict(y=dev(torch, ys[i]), hx=probs[i].hr_shape[0], wx=probs[i].hr_shape[1],
                     psf=probs[i].psf, decim=probs[i].decim, sigma=probs[i].sigma,
                     lam=probs[i].lam) for i in idx]

    outs, stats = rb.solve_batch(items([0, 1, 2]))
    for i, (p, y, xo, st) in enumerate(zip(probs, ys, outs, stats)):
        r = Restorer(0).configure(p, precision="bf16", method="rre", L=5, m=0, tol=1e-5,
                                  max_fp_calls=200)
        r.set_precision_switch(1e-4)
        xs, sst = r.solve(dev(torch, y), *p.hr_shape)
        e = rel(host(xo), host(xs))
        say(f"  {p.name}: batched {st['fp_calls']} calls, single {sst['fp_calls']}, {e:.2e}")
        assert st["status"] == 0 and st["fp_calls"] == sst["fp_calls"]
        assert e <= 3e-5
        alone, _ = rb.solve_batch(items([i]))
        assert np.array_equal(host(alone[0]), host(xo))
