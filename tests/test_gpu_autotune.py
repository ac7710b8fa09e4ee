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
    c = api.get_config("md_run", n, "fp64")
    assert c["tuned"]
    print(f"[autotune n={n}] {c}", flush=True)
    d = inputs.cloud1024(n=n, seed=3)
    F = np.stack([t.cpu().numpy() for t in api.coulomb_forces(*[dev(d[k]) for k in ("x", "y", "z", "q")])])
    ref = np.stack(oracle.forces(d["x"], d["y"], d["z"], d["q"]))
    assert per_ion_rel(F, ref).max() <= 1e-12
    for op in ("forces", "md_step", "md_run"):
        api.reset_config(op, n, "fp64")
    assert not api.get_config("forces", n, "fp64")["tuned"]
    api.load_tuning(cache)
    c2 = api.get_config("forces", n, "fp64")
    assert c2["tuned"] and (c2["algo"], c2["p"], c2["splits"]) == (c["algo"], c["p"], c["splits"])
    api.autotune("hvp", 2000, "fp64")
    assert api.get_config("adjoint", 2000, "fp64")["tuned"]
    for op in ("forces", "md_step", "md_run"):
        api.reset_config(op, n, "fp64")
    api.reset_config("hvp", 2000, "fp64")
    api.reset_config("adjoint", 2000, "fp64")
