"""GPU autotuner: picks a configuration, results stay correct, the cache
round-trips."""
import numpy as np
import pytest

from paper_2106_11143_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_11143_amd import api as A
    A.lib()
    return A


def test_autotune_roundtrip(api, oracle, tmp_path):
    from _gpu_util import dev, per_ion_rel
    n = 6000
    cache = str(tmp_path / "tune.jsonl")
    api.autotune("forces", n, "fp64", cache)
    assert api.get_config("forces", n, "fp64")["tuned"]
    # at n <= 8192 tuning the forces leaves md_step / md_run alone; tuning
    # md_run times whole steps (two-launch step or one-launch step)
    assert not api.get_config("md_run", n, "fp64")["tuned"]
    api.autotune("md_run", n, "fp64", cache)
    cm = api.get_config("md_run", n, "fp64")
    assert cm["tuned"] and api.get_config("md_step", n, "fp64") == cm
    c = api.get_config("forces", n, "fp64")
    assert c["tuned"]
    print(f"[autotune n={n}] forces {c} md_run {cm}", flush=True)
    d = inputs.cloud1024(n=n, seed=3)
    F = np.stack([t.cpu().numpy() for t in api.coulomb_forces(*[dev(d[k]) for k in ("x", "y", "z", "q")])])
    ref = np.stack(oracle.forces(d["x"], d["y"], d["z"], d["q"]))
    assert per_ion_rel(F, ref).max() <= 1e-12
    for op in ("forces", "md_step", "md_run"):
        api.reset_config(op, n, "fp64")
    assert not api.get_config("forces", n, "fp64")["tuned"]
    assert not api.get_config("md_run", n, "fp64")["tuned"]
    api.load_tuning(cache)  # the later lines of the cache win
    c2 = api.get_config("forces", n, "fp64")
    assert c2["tuned"] and (c2["algo"], c2["p"], c2["splits"]) == (c["algo"], c["p"], c["splits"])
    assert api.get_config("md_run", n, "fp64") == cm
    d2 = inputs.cloud1024(n=n, seed=4)  # the tuned one-launch step against the oracle
    st = inputs.state9(d2)
    ts = [dev(st[k]) for k in range(9)]
    api.md_run(ts, dev(d2["q"]), dev(d2["m"]), d2["trap"], 0.0, d2["dt"], 3)
    ref, _, _ = oracle.md_run(st, d2["q"], d2["m"], d2["trap"], 0.0, d2["dt"], 3)
    got = np.stack([t.cpu().numpy() for t in ts])
    for blk in (slice(0, 3), slice(3, 6), slice(6, 9)):
        assert np.abs(got[blk] - ref[blk]).max() <= 1e-11 * np.abs(ref[blk]).max()
    api.autotune("hvp", 2000, "fp64")
    assert api.get_config("adjoint", 2000, "fp64")["tuned"]
    for op in ("forces", "md_step", "md_run"):
        api.reset_config(op, n, "fp64")
    api.reset_config("hvp", 2000, "fp64")
    api.reset_config("adjoint", 2000, "fp64")
