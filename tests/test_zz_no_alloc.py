"""coulomb_forces_noalloc (the allocation-free variant of coulomb_forces, its
partial sums in the library's static per-GPU scratch) against
coulomb_forces, called through the C ABI: two calls in a row, the second on
a smaller input, on both of its paths (the Newton's-third-law stage when its
tiles fit in the scratch, else the all-pairs kernel with its j-splits capped
to the scratch)."""
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


def _cloud(n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    return dict(x=g.normal(0, 150e-6, n), y=g.normal(0, 150e-6, n), z=g.normal(0, 800e-6, n),
                q=inputs.E_CHARGE * g.choice([1.0, 2.0], n, p=[0.99, 0.01]))


# (first n, second n): the scratch's Newton's-third-law path (<= ~32768 ions),
# the capped all-pairs path (larger), both orders, ragged and tiny sizes
SEQUENCES = [(100000, 32768), (32768, 20001), (65537, 4097), (20000, 1), (3000, 2)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n1,n2", SEQUENCES)
def test_noalloc_matches_coulomb_forces(api, prec, n1, n2):
    import torch
    from _gpu_util import dev
    for call, n in enumerate((n1, n2)):
        d = _cloud(n, 500 + n)
        args = [dev(d[k]) for k in "xyzq"]
        ref = torch.stack(api.coulomb_forces(*args, prec=prec))
        out = tuple(torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3))
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        res = api.coulomb_forces_noalloc(*args, prec=prec, out=out)
        torch.cuda.synchronize()
        after = torch.cuda.memory_allocated()
        assert after == before, (before, after)  # the call took no torch memory
        got = torch.stack(res)
        del res
        cfg = api.get_config("forces", n, prec)
        if n == 1:
            assert bool((got == 0).all())
            continue
        err = (torch.linalg.norm(got - ref, dim=0) / torch.linalg.norm(ref, dim=0)).max().item()
        print(f"[noalloc {prec} call {call} n={n} algo={cfg['algo']}] max rel vs coulomb_forces {err:.3e}",
              flush=True)
        assert err <= (1e-12 if prec == "fp64" else 1e-7), (n, err)
        if cfg["algo"] in (1, 2) and n <= 32768:
            assert torch.equal(got, ref)  # the same stage in the scratch: bitwise
    assert api.poll_flags() == 0


def test_noalloc_rejects_beyond_scratch(api):
    from _gpu_util import dev
    n = 2796203  # one more ion than the 64 MiB scratch holds at 24 bytes per ion
    x = dev(np.zeros(1))
    L = api.lib()
    st = L.coulomb_forces_noalloc(n, x.data_ptr(), x.data_ptr(), x.data_ptr(), x.data_ptr(), 0.0, 0,
                                  x.data_ptr() + 8, x.data_ptr() + 16, x.data_ptr() + 24, None)
    assert st == api.CB_ENOWS
    assert "scratch" in api.last_error()
