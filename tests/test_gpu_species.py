"""Ions grouped by species (contiguous runs of one charge; the paper's
section 2 splits a two-species problem into single-species N-body
sub-problems): tiles and j-ranges of one charge per side take the
charge-free pair loops, tiles across a species boundary the general loop.
Every layout is checked against the oracle, which keeps per-ion charges."""
import numpy as np
import pytest

from paper_2106_11143_amd import inputs

pytestmark = pytest.mark.gpu
E = inputs.E_CHARGE
M40 = inputs.MASS_40U


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_11143_amd import api as A
    A.lib()
    return A


def _charges(n, layout, g):
    if layout == "uniform":
        return np.full(n, E)
    if layout == "uniform_neg":
        return np.full(n, -2.0 * E)
    if layout == "two":  # a boundary inside a block and a segment
        q = np.full(n, E)
        q[int(0.37 * n):] = 2.0 * E
        return q
    if layout == "three":
        q = np.full(n, E)
        q[n // 3:2 * n // 3] = -E
        q[2 * n // 3:] = 3.0 * E
        return q
    return E * g.choice([1.0, 2.0, -1.0], n)  # "random": the general loop everywhere


def _cloud(n, seed, layout):
    g = np.random.Generator(np.random.PCG64(seed))
    return dict(x=g.normal(0, 20e-6, n), y=g.normal(0, 20e-6, n), z=g.normal(0, 60e-6, n), q=_charges(n, layout, g))


def _forces(api, d, prec, eps2=0.0):
    from _gpu_util import dev, host
    return np.stack([host(t) for t in api.coulomb_forces(*(dev(d[k]) for k in "xyzq"), eps2=eps2, prec=prec)])


LAYOUTS = ["uniform", "uniform_neg", "two", "three", "random"]
SIZES = [2, 3, 65, 129, 513, 1000, 2049, 4001]
# (algo, p, wg, splits): direct kernel shapes, then Newton's-third-law shapes
SHAPES = [(0, 1, 64, 1), (0, 2, 128, 7), (0, 4, 256, 64), (1, 2, 4, 256), (2, 4, 4, 512), (2, 8, 4, 512),
          (1, 6, 4, 1024), (2, 3, 4, 256), (4, 4, 4, 256), (4, 8, 4, 512)]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("algo,p,wg,splits", SHAPES)
def test_species_layouts_ragged_sizes(api, oracle, layout, algo, p, wg, splits):
    from _gpu_util import per_ion_rel
    for n in SIZES:
        d = _cloud(n, 4000 + n, layout)
        eps2 = (1e-7) ** 2 if n % 2 else 0.0
        ref = np.stack(oracle.forces(d["x"], d["y"], d["z"], d["q"], eps2=eps2))
        for prec in ("fp64", "mixed"):
            api.set_config("forces", n, prec, p=p, wg=wg, splits=splits, algo=algo)
            try:
                F = _forces(api, d, prec, eps2)
            finally:
                api.reset_config("forces", n, prec)
            err = per_ion_rel(F, ref)
            assert err.max() <= (1e-12 if prec == "fp64" else 1e-7), (layout, n, prec, err.max())
            if algo:
                assert np.linalg.norm(F.sum(axis=1)) <= 1e-13 * np.linalg.norm(F, axis=0).sum()
    api.clear_workspace_cache()


@pytest.mark.parametrize("n", [16384, 33000])
@pytest.mark.parametrize("layout", ["uniform", "two", "three"])
def test_species_default_launch(api, oracle, layout, n):
    """Default launches at sizes that take the Newton's-third-law stage with
    P = 4 (JL 256) and P = 8 (JL 512)."""
    from _gpu_util import per_ion_rel, report
    d = _cloud(n, 5000 + n, layout)
    fx, fy, fz, kappa = oracle.forces(d["x"], d["y"], d["z"], d["q"], kappa=True)
    ref = np.stack([fx, fy, fz])
    for prec in ("fp64", "mixed"):
        err = per_ion_rel(_forces(api, d, prec), ref)
        report(f"species {layout} n={n} {prec}", err, kappa)
        assert err.max() <= (1e-12 if prec == "fp64" else 1e-7)


@pytest.mark.parametrize("layout", ["uniform", "two", "random"])
@pytest.mark.parametrize("n", [2, 777, 5000])
def test_species_energy(api, oracle, layout, n):
    from _gpu_util import dev
    d = _cloud(n, 6000 + n, layout)
    ref, _ = oracle.coulomb_energy(d["x"], d["y"], d["z"], d["q"])
    for prec, tol in (("fp64", 1e-12), ("mixed", 1e-9)):
        u = float(api.coulomb_energy(*(dev(d[k]) for k in "xyzq"), prec=prec)[0])
        assert abs(u - ref) <= tol * abs(ref), (layout, n, prec, u, ref)


@pytest.mark.parametrize("n", [1000, 20000])
def test_species_md_run_matches_oracle(api, oracle, n):
    """Two species grouped (a boundary inside a block), md_run with energies,
    on the direct (1000 ions) and Newton's-third-law (20000) paths."""
    from _gpu_util import dev, state_host, state_tensors
    d = _cloud(n, 7000 + n, "two")
    st = np.zeros((9, n))
    st[:3] = np.stack([d["x"], d["y"], d["z"]])
    st[3:6] = inputs.maxwell(np.random.Generator(np.random.PCG64(n)), n, 10e-3, M40)
    m = np.full(n, M40)
    m[int(0.37 * n):] *= 2.0
    trap = inputs.pseudo_trap(1e6, 1e6, 0.2e6)
    nsteps, every = (20, 5) if n <= 1000 else (5, 5)
    ref, en_ref, _ = oracle.md_run(st, d["q"], m, trap, 0.0, 1e-9, nsteps, every=every)
    perm = np.arange(n)[::-1]
    alt, en_alt, _ = oracle.md_run(st[:, perm], d["q"][perm], m[perm], trap, 0.0, 1e-9, nsteps, every=every)
    alt = alt[:, np.argsort(perm)]
    ts = state_tensors(st)
    en = api.md_run(ts, dev(d["q"]), dev(m), trap, 0.0, 1e-9, nsteps, every=every)
    got = state_host(ts)
    for blk in (slice(0, 3), slice(3, 6), slice(6, 9)):
        D = np.abs(alt[blk] - ref[blk]).max()
        assert np.abs(got[blk] - ref[blk]).max() <= 10 * D + 1e-13 * np.abs(ref[blk]).max(), blk
    en = en.cpu().numpy()[0]
    assert np.all(np.abs(en - en_ref) <= 10 * np.abs(en_alt - en_ref) + 1e-12 * np.abs(en_ref).max(axis=0))


@pytest.mark.parametrize("path", [("stepped", 4, 256), ("stepped", 8, 512), ("persistent",)],
                         ids=lambda p: "-".join(map(str, p)))
def test_species_ensemble_matches_oracle(api, oracle, path):
    """Ensemble runs of one species each (different charges per run) and runs
    of two grouped species, on both ensemble paths, run by run."""
    from _gpu_util import dev
    sizes = [300, 1100, 64, 700]
    layouts = ["uniform", "two", "uniform_neg", "three"]
    g = np.random.Generator(np.random.PCG64(71))
    trap = inputs.pseudo_trap(1.0e6, 1.0e6, 0.15e6)
    parts, qs = [], []
    for n, lay in zip(sizes, layouts):
        sig = inputs.crystal_sigma(n, trap["wx"], trap["wy"], trap["wz"])
        st = np.zeros((9, n))
        st[:3] = g.normal(size=(3, n)) * sig[:, None]
        st[3:6] = inputs.maxwell(g, n, 10e-3, M40)
        parts.append(st)
        q = np.abs(_charges(n, lay, g)) if lay != "uniform_neg" else _charges(n, lay, g)
        qs.append(q)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    st = np.concatenate(parts, axis=1)
    q = np.concatenate(qs)
    m = np.full(offs[-1], M40)
    ntot = int(offs[-1])
    if path[0] == "persistent":
        api.set_config("md_ensemble", ntot, "fp64", p=4, wg=512, splits=1, algo=0)
    else:
        api.set_config("md_ensemble", ntot, "fp64", p=path[1], wg=4, splits=path[2], algo=2)
    try:
        ts = [dev(st[k]) for k in range(9)]
        api.md_run(ts, dev(q), dev(m), [trap] * len(sizes), 0.0, 1e-9, 12, offsets=offs)
        got = np.stack([t.cpu().numpy() for t in ts])
    finally:
        api.reset_config("md_ensemble", ntot, "fp64")
    for r in range(len(sizes)):
        sl = slice(offs[r], offs[r + 1])
        ref, _, _ = oracle.md_run(parts[r], q[sl], m[sl], trap, 0.0, 1e-9, 12)
        perm = np.arange(sizes[r])[::-1]
        alt, _, _ = oracle.md_run(parts[r][:, perm], q[sl][perm], m[sl][perm], trap, 0.0, 1e-9, 12)
        alt = alt[:, np.argsort(perm)]
        for blk in (slice(0, 3), slice(3, 6), slice(6, 9)):
            D = np.abs(alt[blk] - ref[blk]).max()
            err = np.abs(got[blk, sl] - ref[blk]).max()
            assert err <= 10 * D + 1e-13 * np.abs(ref[blk]).max(), (r, blk, err, D)


@pytest.mark.parametrize("algo,p,wg,splits", [(0, 1, 64, 1), (2, 4, 4, 256)])
def test_nonfinite_charge_reaches_the_forces(api, algo, p, wg, splits):
    """A NaN charge in an otherwise uniform range must not be skipped by the
    charge-free loop: the forces it touches are NaN and the flag is set."""
    n = 3000
    d = _cloud(n, 8000, "uniform")
    d["q"] = d["q"].copy()
    d["q"][2500] = np.nan
    api.poll_flags()
    api.set_config("forces", n, "fp64", p=p, wg=wg, splits=splits, algo=algo)
    try:
        F = _forces(api, d, "fp64")
    finally:
        api.reset_config("forces", n, "fp64")
    assert api.poll_flags() & 1
    assert np.isnan(F[:, 0]).any() and np.isnan(F[:, 2500]).any()


def test_cloud100k_grouped_by_species(api, oracle):
    """The headline cloud with its ions relabelled so that the +2e ions come
    last (the same system): sampled ions against the oracle, Newton's third
    law on the whole result, and the ungrouped order's forces relabelled."""
    from _gpu_util import dev, host, per_ion_rel, report
    d = inputs.cloud100k()
    dg = inputs.group_by_charge(d)
    n = d["n"]
    assert np.all(np.diff(dg["q"]) >= 0) and np.array_equal(np.sort(d["q"]), dg["q"])
    F = np.stack([host(t) for t in api.coulomb_forces(*(dev(dg[k]) for k in "xyzq"))])
    g = np.random.Generator(np.random.PCG64(91))
    idx = np.unique(np.concatenate([np.arange(n - 1100, n - 900), g.choice(n, 800, replace=False)]))
    fx, fy, fz, kappa = oracle.forces(dg["x"], dg["y"], dg["z"], dg["q"], idx=idx, kappa=True)
    err = per_ion_rel(F[:, idx], np.stack([fx, fy, fz]))
    report("cloud100k grouped (sampled)", err, kappa)
    assert err.max() <= 1e-12
    assert np.linalg.norm(F.sum(axis=1)) <= 1e-12 * np.linalg.norm(F, axis=0).sum()
    Fu = np.stack([host(t) for t in api.coulomb_forces(*(dev(d[k]) for k in "xyzq"))])
    e = per_ion_rel(F, Fu[:, dg["perm"]])
    assert e.max() <= 1e-12
