"""GPU: the autotuner's search (every candidate must return identical bits,
checked inside the library), its choice against the oracle, and the JSON
cache."""
import numpy as np
import pytest

import oracle
from paper_1108_3126_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_tune_single_fixed_and_offsets(dev, tmp_path):
    from paper_1108_3126_amd import autotune, rx

    prog = W.single_program(1)
    s, _ = W.single_strings(prog, seed=31, n=6000, length=64)
    want = oracle.match(prog.ast, prog.root, prog.classes, True, s.data, s.offsets)
    p = rx.compile(prog.ast, prog.root, prog.classes, True).upload(dev).jit()
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    cache = str(tmp_path / "tune.json")
    best, info = autotune.tune_single(p, d, length=64, cache_path=cache)
    print("tuned fixed:", info, flush=True)
    assert info["candidates"] >= 10 and not info["cached"]
    got = rx.match_fixed(p, d, 64, s.n, launch=best).cpu().numpy()
    assert np.array_equal(got, want)
    best2, info2 = autotune.tune_single(p, d, length=64, cache_path=cache)
    assert info2["cached"] and (best2.variant, best2.block, best2.grid) == (best.variant, best.block, best.grid)
    best3, info3 = autotune.tune_single(p, d, offsets=o, cache_path=cache)
    print("tuned offsets:", info3, flush=True)
    assert np.array_equal(rx.match(p, d, o, launch=best3).cpu().numpy(), want)


def test_tune_multi(dev, tmp_path):
    from paper_1108_3126_amd import autotune, rx

    progs = W.multi_programs(seed=5, count=4, lo=16, hi=200)
    s = W.multi_lines(seed=5, n=2500, hi=900)
    want = np.stack([oracle.match(p.ast, p.root, p.classes, True, s.data, s.offsets) for p in progs])
    ps = [rx.compile(p.ast, p.root, p.classes, True).upload(dev) for p in progs]
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    cfg, info = autotune.tune_multi(ps, d, o, budget_runs=40, cache_path=str(tmp_path / "t.json"))
    print("tuned multi:", info, flush=True)
    assert info["candidates"] == 27
    assert np.array_equal(rx.match_multi(ps, d, o, config=cfg).cpu().numpy(), want)


def test_tune_multi_with_plane_form(dev, tmp_path):
    """With the list prepared, the tuner also times the plane form; whatever wins gives the oracle's bits."""
    from paper_1108_3126_amd import autotune, rx

    progs = W.multi_programs(seed=6, count=3, lo=16, hi=200)
    s = W.multi_lines(seed=6, n=6000, hi=900)
    want = np.stack([oracle.match(p.ast, p.root, p.classes, True, s.data, s.offsets) for p in progs])
    ps = [rx.compile(p.ast, p.root, p.classes, True).upload(dev) for p in progs]
    rx.prepare_multi(ps)
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    cfg, info = autotune.tune_multi(ps, d, o, budget_runs=40, cache_path=str(tmp_path / "t.json"), planes=True)
    print("tuned multi with planes:", info, flush=True)
    assert info["candidates"] == 28
    assert np.array_equal(rx.match_multi(ps, d, o, config=cfg).cpu().numpy(), want)
    cfg2, info2 = autotune.tune_multi(ps, d, o, cache_path=str(tmp_path / "t.json"), planes=True)
    assert info2["cached"] and cfg2.form == cfg.form
