"""Launch configurations of the single-image path (redve_set_tuning / redve_set_autotune),
through the C ABI: every valid configuration of the kernels (stage threads, tabulated or
windowed influence functions, one or two CG iterations per launch, one-iteration CG threads,
the CG start formed by the last stage or by its own kernel) computes one FP call of eq. (7)
within its bar of the FP64 oracle, on an image below and one above the 512-tile size where the
built-in rules switch; the autotuner picks one of them, caches it in its JSON lines file, and
a new handle reading that file uses it without tuning again."""
import itertools
import json

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


FIELDS = ("stage_threads", "phi_table", "cg_per_launch", "cg_threads", "fused_start", "cg_tile")


def valid_configs(r, hx, wx):
    """Every configuration the library accepts and resolves to itself for this image."""
    from paper_1805_02158_amd import RedveError
    out = []
    for v in itertools.product((512, 1024), (1, 2), (1, 2), (256, 1024), (1, 2), (16, 32)):
        cfg = dict(zip(FIELDS, v))
        try:
            r.set_tuning(cfg)
        except RedveError:
            continue
        got, us = r.get_tuning(hx, wx)
        assert us == -1.0
        if got == cfg:
            out.append(cfg)
    r.set_tuning(None)
    return out


def sized(h, w, seed):
    return W.Problem(f"u9_{h}x{w}", W.make_image(h, w, seed), W.psf_uniform(9), 1, W.SQRT2, 0.02,
                     W.make_noise((h, w), seed + 100), 15, W.make_denoiser())


# 256x256: 256 tiles (rules: 1024 threads, tables, two CG iterations per launch, fused start);
# 400x330: 525 tiles (rules: 512 threads, window, one iteration per launch)
@pytest.mark.parametrize("name", ["deblur256", "400x330"])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_every_configuration_matches_the_oracle(torch, orc, name, precision):
    from paper_1805_02158_amd import Restorer
    prob = W.problem("deblur256") if name == "deblur256" else sized(400, 330, 1950)
    hx, wx = prob.hr_shape
    op = orc.OracleProblem(prob, y=f32(orc.OracleProblem(prob).y))
    x = f32(op.y)
    xo = op.fp(x)
    r = Restorer(0).configure(prob, precision=precision)
    cfgs = valid_configs(r, hx, wx)
    say(f"{name} {precision}: {len(cfgs)} configurations")
    assert len(cfgs) >= 4
    results = []
    for cfg in cfgs:
        r.set_tuning(cfg)
        xg = host(r.fp_step(dev(torch, op.y), dev(torch, x)))
        e, es = rel(xg, xo), rel(xg - x, xo - x)
        say(f"  {cfg}: rel L2 {e:.2e}, relative to the step {es:.2e}")
        if precision == "fp32":
            assert e <= 2e-5 and es <= 1e-4
        else:  # BF16 filter-bank operands: the update carries their 3.9e-3 relative error
            assert e <= 2e-4 and es <= 5e-3
        results.append(xg)
    if precision == "fp32":  # the same arithmetic in every configuration but rounding order
        for xg in results[1:]:
            assert rel(xg, results[0]) <= 2e-6


def test_autotune_picks_caches_and_reuses(torch, orc, tmp_path):
    from paper_1805_02158_amd import Restorer
    prob = W.problem("deblur256")
    hx, wx = prob.hr_shape
    y32 = f32(orc.OracleProblem(prob).y)
    cache = tmp_path / "tuning.jsonl"
    r = Restorer(0).configure(prob, precision="bf16", method="rre", L=5, tol=1e-5,
                              max_fp_calls=100)
    r.set_autotune(True, str(cache))
    cfg0, us0 = r.get_tuning(hx, wx)
    assert us0 == -1.0  # not tuned yet: the rules
    x, st = r.solve(dev(torch, y32), hx, wx)
    cfg, us = r.get_tuning(hx, wx)
    say(f"  tuned {cfg} at {us:.1f} us per FP call (rules: {cfg0})")
    assert us > 0 and cfg in valid_configs(Restorer(0).configure(prob, precision="bf16"), hx, wx)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    entry = json.loads(lines[0])
    assert entry["key"][:2] == [hx, wx] and all(entry[k] == cfg[k] for k in cfg)
    # the converged result is the oracle's fixed point within the BF16 bar
    ref = orc.solve(orc.OracleProblem(prob, y=y32), "rre", L=5, m=0, tol=1e-10, max_calls=300)
    assert rel(host(x), ref.x) <= 5e-3
    # a new handle reads the cache and uses the entry without tuning again
    r2 = Restorer(0).configure(prob, precision="bf16", method="rre", L=5, tol=1e-5,
                               max_fp_calls=100)
    r2.set_autotune(True, str(cache))
    cfg2, us2 = r2.get_tuning(hx, wx)
    assert cfg2 == cfg and abs(us2 - us) < 1e-3 * us
    x2, _ = r2.solve(dev(torch, y32), hx, wx)
    assert len(cache.read_text().splitlines()) == 1
    assert np.array_equal(host(x2), host(x))


@pytest.mark.parametrize("shape", [(37, 53), (100, 70), (2, 3), (400, 330), (520, 512)])
@pytest.mark.parametrize("psf", ["u9", "g7"])
@pytest.mark.parametrize("tile", [16, 32])
def test_cg_forms_match_the_oracle(torch, orc, shape, psf, tile):
    """CG on A x = rhs against the oracle's CG with the one-iteration kernel forced to 16x16
    tiles (r, A r, A p, p, d in HBM) or 32x32 tiles (r, p, d only; A r and A p recomputed on
    halos of 2 x 8 or 2 x 6 pixels): images smaller than one tile and than the halo (periodic
    wrap), ragged tiles, and images of more than 512 16x16 tiles, 1 to 15 iterations."""
    from paper_1805_02158_amd import Restorer
    k = W.psf_uniform(9) if psf == "u9" else W.psf_gaussian(7, 1.6)
    r = Restorer(0)
    r.set_operator(k, 1).set_noise(2 ** 0.5).set_lambda(0.02)
    r.set_tuning({"cg_per_launch": 1, "cg_tile": tile})
    got, _ = r.get_tuning(*shape)
    assert got["cg_tile"] == tile
    rng = np.random.default_rng(9)
    x0 = f32(rng.uniform(0, 255, shape))
    rhs = f32(orc.apply_A(rng.uniform(0, 255, shape), k, 1, 2 ** 0.5, 0.02))
    for iters in (1, 2, 3, 15):
        xg = host(r.cg(dev(torch, rhs), dev(torch, x0), iters))
        xo = orc.cg(rhs, x0, f32(k), 1, 2 ** 0.5, 0.02, iters)
        e = rel(xg, xo)
        say(f"  {shape} {psf} tile {tile} iters {iters}: rel L2 {e:.2e}")
        assert e <= 2e-5, iters
